"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs, element by element, through the C ABI.

Tolerance (FP64 path): 1e-12, the target stated for the steady profiles;
populations are compared relative to the largest population of their cell,
n and T relative, u relative to the thermal speed sqrt(T_left/m)."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import compare, initial_states, oracle_dt, run_gpu, run_oracle  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1708_03249_amd as H
    H.lib()


def H():
    import paper_1708_03249_amd as H
    return H


def _check(channels, nsteps, perturb=0.0, seed=0, tol=TOL, which=None, what="", tuning=None):
    print(f"[parity] {what}: {len(channels)} channels, {nsteps} steps", flush=True)
    states = initial_states(channels, seed=seed, perturb=perturb)
    gpu = run_gpu(channels, states, nsteps, tuning=tuning)
    assert gpu["bad"] == 0
    ref = run_oracle(channels, states, nsteps, gpu["dt"], which=which)
    return compare(channels, gpu, ref, tol=tol, what=what)


def test_small_channel_upwind3():
    """HHLB(3;4), Nx = 64 (two windows, the second ragged), third-order
    upwind, equal walls, Kn = 0.1, g = -0.1, dt = 5e-4."""
    h = H()
    ch = h.Channel(quad=h.HALF_HERMITE, Q=4, Nx=64, adv=h.UPWIND3, transverse_dof=2, Kn=0.1,
                   g=-0.1, dt=5e-4)
    _check([ch], 400, what="small upwind3")


def test_stretched_weno5_three_kn_batched():
    """HHLB(7;8), tanh-stretched grid A = 0.9, WENO-5, T_left = 1, T_right = 2,
    g = -0.5, Kn in {0.01, 0.1, 1} as three channels of one solver, CFL 0.5,
    perturbed start (exercises the non-linear WENO weights)."""
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=8, Nx=200, adv=h.WENO5, stretch_A=0.9,
                       T_left=1.0, T_right=2.0, g=-0.5, Kn=kn, dt=-0.5) for kn in (0.01, 0.1, 1.0)]
    _check(chans, 60, perturb=0.05, what="stretched weno5")


def test_full_range_hlb16():
    """HLB(15;16) (full-range Gauss-Hermite comparison model), stretched grid."""
    h = H()
    ch = h.Channel(quad=h.FULL_HERMITE, Q=16, Nx=130, adv=h.WENO5, stretch_A=0.9, T_left=1.0,
                   T_right=2.0, g=-0.5, Kn=0.1, dt=-0.5)
    _check([ch], 60, perturb=0.02, what="HLB(15;16)")


def test_q16_weno5():
    """HHLB(15;16), V = 32, the node count of the large workload."""
    h = H()
    ch = h.Channel(quad=h.HALF_HERMITE, Q=16, Nx=150, adv=h.WENO5, stretch_A=0.9, T_left=1.0,
                   T_right=1.5, g=-1.0, Kn=0.02, dt=-0.5)
    _check([ch], 25, perturb=0.02, what="HHLB(15;16)")


def test_half_range_laguerre():
    """Half-range Gauss-Laguerre model (Eqs. wk_half, hh_Kk_L) through the same
    kernels: Q = 4 upwind-3 (two windows, ragged), Q = 8 WENO-5 on the
    stretched grid with a perturbed start, Q = 16 WENO-5 (matrix-core path),
    p0 scaled so the nodes span the thermal range."""
    h = H()
    chans = [h.Channel(quad=h.HALF_LAGUERRE, Q=4, Nx=64, adv=h.UPWIND3, transverse_dof=2, Kn=0.1,
                       g=-0.3, T_left=1.0, T_right=1.4, p0=0.4, dt=-0.5),
             h.Channel(quad=h.HALF_LAGUERRE, Q=8, Nx=130, adv=h.WENO5, stretch_A=0.9, Kn=0.05,
                       g=-0.5, T_left=1.0, T_right=2.0, p0=0.3, dt=-0.5),
             h.Channel(quad=h.HALF_LAGUERRE, Q=16, Nx=121, adv=h.WENO5, stretch_A=0.6, Kn=0.02,
                       g=-1.0, T_left=1.0, T_right=1.5, p0=0.2, dt=-0.5)]
    _check(chans, 40, perturb=0.03, what="half-range Laguerre")


def test_large_q_node_parallel():
    """Q > 16 (the node-parallel stage): HHLB(19;20) WENO-5 with chi over two
    windows (the second ragged) on a stretched grid with a perturbed start;
    HHLB(12;17) upwind-3 with N < Q-1; HHLB(20;40) collisionless."""
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=20, N=19, Nx=70, adv=h.WENO5, transverse_dof=2,
                       stretch_A=0.8, Kn=0.05, g=-0.5, T_left=1.0, T_right=1.6, dt=-0.5),
             h.Channel(quad=h.HALF_HERMITE, Q=17, N=12, Nx=59, adv=h.UPWIND3, transverse_dof=2,
                       Kn=0.2, g=0.3, T_left=1.2, T_right=1.0, dt=-0.5),
             h.Channel(quad=h.HALF_HERMITE, Q=40, N=20, Nx=24, adv=h.WENO5, transverse_dof=0,
                       stretch_A=0.9, Kn=math.inf, g=0.1, T_left=1.4, T_right=0.6, dt=-0.5)]
    _check(chans, 20, perturb=0.03, what="large Q")


def test_large_q_launch_configurations_identical():
    """The node-parallel path gives the same bits with and without the
    XCD-aware block mapping, with direct launches and with graph replay of
    several lengths (each block computes the same values whatever its
    position in the grid)."""
    import torch
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=24, N=20, Nx=150, adv=h.WENO5, transverse_dof=2,
                       stretch_A=0.7, Kn=0.1, g=-0.3, T_left=1.0, T_right=1.3, dt=-0.5),
             h.Channel(quad=h.HALF_HERMITE, Q=40, N=20, Nx=70, adv=h.UPWIND3, transverse_dof=0,
                       Kn=math.inf, g=0.2, T_left=1.2, T_right=0.9, dt=-0.5)]
    states = initial_states(chans, seed=3)
    f0 = torch.from_numpy(np.concatenate([st[0].ravel() for st in states])).cuda()
    c0 = torch.from_numpy(np.concatenate([st[1].ravel() for st in states])).cuda()
    configs = [dict(), dict(xcd_map=0), dict(graph_steps=16, xcd_map=1), dict(graph_steps=3, xcd_map=0)]
    outs = []
    for cfg in configs:
        s = h.Solver(chans)
        s.set_tuning(**cfg)
        s.set_state(f0, c0)
        s.step(5)
        s.step(6)
        f, c = s.get_state()
        torch.cuda.synchronize()
        outs.append((f.cpu().numpy(), c.cpu().numpy()))
        s.close()
    assert np.all(np.isfinite(outs[0][0]))
    for k in range(1, len(outs)):
        assert np.array_equal(outs[0][0], outs[k][0]), configs[k]
        assert np.array_equal(outs[0][1], outs[k][1]), configs[k]


def test_full_range_large_q_node_parallel():
    """Full-range HLB(N;Q) with Q > 16 (the node-parallel stage, dense force
    contraction over all V = Q rows): HLB(20;40) WENO-5 with chi on a
    stretched grid with a perturbed start, HLB(19;24) upwind-3, and
    HLB(20;100) collisionless from a smooth start."""
    h = H()
    chans = [h.Channel(quad=h.FULL_HERMITE, Q=40, N=20, Nx=70, adv=h.WENO5, transverse_dof=2,
                       stretch_A=0.8, Kn=0.05, g=-0.5, T_left=1.0, T_right=1.6, dt=-0.5),
             h.Channel(quad=h.FULL_HERMITE, Q=24, N=19, Nx=59, adv=h.UPWIND3, transverse_dof=0,
                       Kn=0.2, g=0.3, T_left=1.2, T_right=1.0, dt=-0.5)]
    _check(chans, 20, perturb=0.03, what="full range, large Q")
    ch = h.Channel(quad=h.FULL_HERMITE, Q=100, N=20, Nx=40, adv=h.WENO5, transverse_dof=0,
                   stretch_A=0.9, Kn=math.inf, g=-1.0, T_left=0.7, T_right=1.3, dt=-0.5)
    _check([ch], 20, what="HLB(20;100)")


def test_full_range_hlb_20_500_ballistic_setup():
    """HLB(20;500), the paper's largest full-range model of the ballistic
    study (Sec. V.E), on its grid: Nx = 24, A = 0.99, Kn = inf, g_p = 1,
    T_left = 1.4, T_right = 0.6, dt = 1e-4; 30 steps against the oracle from
    the equilibrium at rest (smooth in p, as for HHLB(20;200))."""
    h = H()
    ch = h.Channel(quad=h.FULL_HERMITE, Q=500, N=20, Nx=24, adv=h.WENO5, transverse_dof=0,
                   stretch_A=0.99, Kn=math.inf, g=-1.0, T_left=1.4, T_right=0.6, dt=1e-4)
    _check([ch], 30, what="HLB(20;500)")


def test_large_q_limits_minimum_grid():
    """The node-parallel path at its limits on the smallest grid (Nx = 8,
    both walls in one window): half-range Q = 256 (one chunk of 16 MFMA
    steps per wave, 16 tiles per half) with chi and BGK, and full-range
    Q = 512 (two chunks, the dense contraction over 512 rows) with BGK.
    The half-range channel takes the paper's dt = 1e-4: its force matrix
    has spectral radius 2.0e3 (the nodes crowd towards p = 0), and at the
    advective CFL step dt |g| rho(K) = 1.2, where the non-normal force
    operator amplifies any last-bit difference tenfold per step."""
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=256, N=20, Nx=8, adv=h.WENO5, transverse_dof=2,
                       stretch_A=0.5, Kn=0.3, g=-0.4, T_left=1.2, T_right=0.9, dt=1e-4),
             h.Channel(quad=h.FULL_HERMITE, Q=512, N=20, Nx=8, adv=h.UPWIND3, transverse_dof=0,
                       Kn=0.5, g=0.3, T_left=0.9, T_right=1.1, dt=-0.5)]
    _check(chans, 5, what="large Q limits, Nx = 8")


def test_ballistic_hhlb_20_200_setup():
    """The paper's ballistic configuration (Sec. V.E): HHLB(20;200), V = 400,
    Nx = 24, A = 0.99, Kn = inf, g = 0.1, T_left = 1.4, T_right = 0.6,
    dt = 1e-4, the 1-D gas (no chi); 40 steps against the oracle from the
    equilibrium at rest.  The start is smooth in p on purpose: at V = 400 the
    force matrix differentiates like a 400-point spectral operator, so a
    start perturbed at random node by node gives force terms 1e6 times the
    populations and compares rounding orders rather than the method."""
    h = H()
    ch = h.Channel(quad=h.HALF_HERMITE, Q=200, N=20, Nx=24, adv=h.WENO5, transverse_dof=0,
                   stretch_A=0.99, Kn=math.inf, g=0.1, T_left=1.4, T_right=0.6, dt=1e-4)
    _check([ch], 40, what="HHLB(20;200)")


def test_edge_cases_batch():
    """Minimum Nx = 8 (both walls in one window), collisionless Kn = inf,
    no chi (Dt = 0), N < Q - 1, p0 != 1, positive g, a mixed batch of model
    classes in one solver."""
    h = H()
    chans = [
        h.Channel(quad=h.HALF_HERMITE, Q=6, N=3, Nx=8, adv=h.WENO5, transverse_dof=0,
                  Kn=math.inf, g=0.3, p0=1.2, T_left=1.2, T_right=0.8, dt=2e-4),
        h.Channel(quad=h.HALF_HERMITE, Q=1, N=0, Nx=59, adv=h.UPWIND3, transverse_dof=0,
                  Kn=0.3, g=-0.2, dt=1e-3),
        h.Channel(quad=h.HALF_HERMITE, Q=2, Nx=116, adv=h.WENO5, transverse_dof=0, Kn=0.05,
                  g=-0.7, T_right=1.3, dt=-0.4),
        h.Channel(quad=h.FULL_HERMITE, Q=4, Nx=117, adv=h.UPWIND3, transverse_dof=0, Kn=0.2,
                  g=-0.2, T_right=1.1, dt=-0.4),
    ]
    _check(chans, 80, perturb=0.03, seed=5, what="edge batch")


def test_equal_walls_fixed_point():
    """g = 0 and equal walls: the wall Maxwellian is a fixed point."""
    h = H()
    ch = h.Channel(quad=h.HALF_HERMITE, Q=8, Nx=100, adv=h.WENO5, stretch_A=0.5, T_left=1.3,
                   T_right=1.3, g=0.0, Kn=0.05, dt=1e-4)
    states = initial_states([ch], T0=1.3)
    gpu = run_gpu([ch], states, 40)
    f = gpu["f"].reshape(ch.V, ch.Nx)
    np.testing.assert_allclose(f, states[0][0], rtol=1e-13, atol=0)
    np.testing.assert_allclose(gpu["nw"][0], [1.0, 1.0], rtol=1e-13)


def test_mass_conservation_long():
    """Exact mass with diffuse walls: sum_i dx_i n_i constant over 3000 steps
    up to rounding.  Each step rounds every population once per stage, a
    relative random walk of order 1e-16 sqrt(V Nx) per step; 1e-12 after 3000
    steps bounds that with margin, while a non-conserving force term (the
    delta term dropped) drifts by about 1e-4 per unit time."""
    h = H()
    ch = h.Channel(quad=h.HALF_HERMITE, Q=8, Nx=300, adv=h.WENO5, stretch_A=0.9, T_left=1.0,
                   T_right=2.0, g=-0.5, Kn=0.05, dt=-0.5)
    states = initial_states([ch])
    gpu = run_gpu([ch], states, 3000)
    assert abs(gpu["mass"][0] - 1.0) < 1e-12


def test_graph_replay_matches_direct_launches():
    """The HIP-graph replay of hhlb_step gives the same bits as direct
    launches: several calls of 7 steps (less than one 16-step graph, so the
    1-step graph runs too) and of 37 steps, with eager reads of the state and
    synchronisations between the calls."""
    import torch
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=8, Nx=200, adv=h.WENO5, stretch_A=0.9,
                       T_left=1.0, T_right=2.0, g=-0.5, Kn=kn, dt=-0.5) for kn in (0.02, 0.5)]
    states = initial_states(chans, seed=3, perturb=0.05)
    f0 = torch.from_numpy(np.concatenate([s[0].ravel() for s in states])).cuda()
    c0 = torch.from_numpy(np.concatenate([s[1].ravel() for s in states])).cuda()
    solvers = []
    for gsteps in (0, 16, 5):
        s = h.Solver(chans)
        s.set_graph_steps(gsteps)
        s.set_state(f0, c0)
        solvers.append(s)
    for rnd, n in enumerate((7, 7, 37, 1, 16)):
        outs = []
        for s in solvers:
            s.step(n)
            f, c = s.get_state()
            torch.cuda.synchronize()
            outs.append((f.cpu().numpy(), c.cpu().numpy()))
        for k in (1, 2):
            assert np.array_equal(outs[0][0], outs[k][0]), f"f differs, call {rnd}, solver {k}"
            assert np.array_equal(outs[0][1], outs[k][1]), f"chi differs, call {rnd}, solver {k}"
    for s in solvers:
        s.close()


def test_small_channel_20000_steps_golden():
    """HHLB(3;4), Nx = 64, third-order upwind, Kn = 0.1, g = -0.1, equal walls,
    dt = 5e-4: 20 000 steps (t = 10, close to the steady flow) against the
    stored oracle result (tests/golden/small_channel_kn0.1_20000.txt, written
    by make_oracle_golden.py from the oracle alone)."""
    from gpu_common import load_golden
    here = os.path.dirname(os.path.abspath(__file__))
    fg, cg, nwg = load_golden(os.path.join(here, "golden", "small_channel_kn0.1_20000.txt"))
    h = H()
    ch = h.Channel(quad=h.HALF_HERMITE, Q=4, N=3, Nx=64, adv=h.UPWIND3, transverse_dof=2,
                   Kn=0.1, g=-0.1, dt=5e-4)
    states = initial_states([ch])
    print("[parity] small channel, 20000 steps", flush=True)
    gpu = run_gpu([ch], states, 20000)
    f = gpu["f"].reshape(ch.V, ch.Nx)
    c = gpu["chi"].reshape(ch.V, ch.Nx)
    ef = np.max(np.abs(f - fg) / np.abs(fg).max(axis=0, keepdims=True))
    ec = np.max(np.abs(c - cg) / np.abs(cg).max(axis=0, keepdims=True))
    en = np.max(np.abs(gpu["nw"][0] / nwg - 1))
    assert max(ef, ec, en) <= TOL, (ef, ec, en)


def test_bench_size_sampled_channels():
    """The benchmark configuration at full size and in its launch shape (256
    channels x Nx = 16384, HHLB(15;16), WENO-5, f and chi, stretched A = 0.9,
    CFL 0.5, direct launches) from the start the benchmark times: the
    equilibrium (1, 0, 1) times the seeded smooth modulation of every
    population row (the seeds of bench.init_developed), built here from the
    oracle's equilibrium.  20 steps of the whole batch on the GPU; channels
    0, 85, 170 and 255 against the oracle, which resolves its own time step
    (checked against the library's)."""
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    import oracle as O
    from gpu_common import to_oracle
    from paper_1708_03249_amd.inputs import smooth_modulation
    chans = bench.workload()
    h = H()
    s = h.Solver(chans)
    which, nsteps = (0, 85, 170, 255), 20
    print(f"[parity] bench size, 256 x 16384, developed start, {nsteps} steps", flush=True)
    feq, _ = O.initial_state(to_oracle(chans[0]))     # every channel starts from the same (1, 0, 1)
    col = torch.from_numpy(np.ascontiguousarray(feq[:, :1])).cuda()
    f = torch.empty(s.total, dtype=torch.float64, device="cuda")
    c = torch.empty_like(f)
    V, Nx = chans[0].V, chans[0].Nx
    for k in range(len(chans)):
        o0, o1 = int(s.offsets[k]), int(s.offsets[k + 1])
        mf = torch.from_numpy(smooth_modulation(2 * k, V, Nx, 0.05)).cuda()
        mc = torch.from_numpy(smooth_modulation(2 * k + 1, V, Nx, 0.05)).cuda()
        f[o0:o1] = (col * mf).reshape(-1)
        c[o0:o1] = (col * mc).reshape(-1)     # chi = (Dt/2) T0 f_eq = f_eq at T0 = 1, Dt = 2
    s.set_state(f, c)
    del f, c
    s.step(nsteps)
    f, c = s.get_state()
    n, u, T = s.moments()
    nw, mass, bad = s.diagnostics()
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    sub = [chans[w] for w in which]
    gpu = dict(f=[], chi=[], n=[], u=[], T=[])
    off, cel = [0], [0]
    for w, ch in zip(which, sub):
        gpu["f"].append(s.channel_view(f, w).cpu().numpy().ravel())
        gpu["chi"].append(s.channel_view(c, w).cpu().numpy().ravel())
        a0, a1 = int(s.cells[w]), int(s.cells[w + 1])
        for k, arr in (("n", n), ("u", u), ("T", T)):
            gpu[k].append(arr[a0:a1].cpu().numpy())
        off.append(off[-1] + ch.V * ch.Nx)
        cel.append(cel[-1] + ch.Nx)
    nwc = nw.cpu().numpy()
    gpu["nw"] = np.array([nwc[w] for w in which])
    for k in ("f", "chi", "n", "u", "T"):
        gpu[k] = np.concatenate(gpu[k])
    gpu["offsets"], gpu["cells"] = np.array(off), np.array(cel)
    dts = [s.dt[w] for w in which]
    s.close()
    del f, c, n, u, T
    torch.cuda.empty_cache()
    states = []
    for w in which:
        states.append((np.ascontiguousarray(feq * smooth_modulation(2 * w, V, Nx, 0.05)),
                       np.ascontiguousarray(feq * smooth_modulation(2 * w + 1, V, Nx, 0.05))))
    ref = run_oracle(sub, states, nsteps, dts, workers=4)
    compare(sub, gpu, ref, tol=TOL, what="bench size, developed start")


def _batch_sample(n=9, steps_nx=None):
    """Channels of the batched workload (PCG64 seed 0 draws), the first n."""
    h = H()
    from paper_1708_03249_amd.inputs import batch_draws
    return [h.Channel(quad=h.HALF_HERMITE, Q=d["Q"], N=d["Q"] - 1, Nx=d["Nx"], adv=h.WENO5,
                      transverse_dof=2, Kn=d["Kn"], g=d["g"], T_right=d["T_right"], dt=-0.5)
            for d in batch_draws(n, 0)]


def test_batched_workload_sample():
    """The first nine channels of the batched workload (uneven Nx, Q in
    {4, 8, 12}, Kn over four decades, dt = min(CFL 0.5, Kn/2)) in one solver,
    30 steps from a perturbed start, against the oracle."""
    chans = _batch_sample(9)
    assert len({c.Q for c in chans}) > 1
    _check(chans, 30, perturb=0.02, seed=11, what="batched sample")


@pytest.mark.parametrize("merge", [1, 2])
def test_batched_sample_one_launch_across_classes(merge):
    """The same sample, its model classes (Q = 4, 8, 12) advanced by one
    launch per stage (merge_classes = 1: a block per window; 2: persistent
    blocks taking windows in turn) and a graph replay, against the oracle;
    the solver reports one launch per stage."""
    h = H()
    chans = _batch_sample(9)
    s = h.Solver(chans)
    assert s.launch_info()[0] == len({c.Q for c in chans})
    s.set_tuning(merge_classes=merge)
    assert s.launch_info()[0] == 1
    for bad in (dict(merge_classes=3), dict(merge_classes=merge, class_streams=1),
                dict(merge_classes=merge, step_fusion=1), dict(merge_classes=merge, waves_per_window=4)):
        with pytest.raises(h.HHLBError) as e:
            s.set_tuning(**bad)
        assert e.value.status == -1, bad
    s.close()
    _check(chans, 30, perturb=0.02, seed=11, what=f"batched sample, merge_classes={merge}",
           tuning=dict(merge_classes=merge, graph_steps=8))


@pytest.mark.parametrize("merge", [1, 2])
def test_one_launch_across_classes_every_group_shape(merge):
    """Launch groups other than the batch's: Q = 16, 12 and 4 with a
    half-range Gauss-Laguerre Q = 8 class (f and chi, WENO-5; the kernel for
    orders up to 16), and Q = 2 and 6 (f only, upwind-3; up to 8), beside a
    full-range channel that keeps its own launch.  The merged launches (and
    graph replay) give the bits of the per-class launches, and the oracle's
    result within the FP64 tolerance."""
    h = H()
    chans = [
        h.Channel(quad=h.HALF_HERMITE, Q=16, Nx=70, adv=h.WENO5, stretch_A=0.9, T_right=1.4, g=-0.5,
                  Kn=0.05, dt=-0.5),
        h.Channel(quad=h.HALF_HERMITE, Q=4, Nx=90, adv=h.WENO5, T_right=1.2, g=-0.2, Kn=0.2, dt=-0.5),
        h.Channel(quad=h.HALF_HERMITE, Q=12, Nx=64, adv=h.WENO5, stretch_A=0.5, g=-1.0, Kn=0.02, dt=-0.5),
        h.Channel(quad=h.HALF_LAGUERRE, Q=8, N=4, Nx=61, adv=h.WENO5, p0=0.3, T_right=1.3, g=-0.3, Kn=0.1,
                  dt=-0.5),
        h.Channel(quad=h.HALF_HERMITE, Q=2, Nx=40, adv=h.UPWIND3, transverse_dof=0, g=-0.3, Kn=0.1, dt=-0.5),
        h.Channel(quad=h.HALF_HERMITE, Q=6, Nx=75, adv=h.UPWIND3, transverse_dof=0, T_right=1.6, Kn=1.0,
                  dt=-0.5),
        h.Channel(quad=h.FULL_HERMITE, Q=8, Nx=50, adv=h.WENO5, T_right=1.3, g=-0.4, Kn=0.1, dt=-0.5),
    ]
    s = h.Solver(chans)
    assert s.launch_info()[0] == 7
    s.set_tuning(merge_classes=merge)
    assert s.launch_info()[0] == 3   # two launch groups and the full-range class
    s.close()
    nsteps = 20
    print(f"[parity] launch groups, merge_classes={merge}: {len(chans)} channels, {nsteps} steps", flush=True)
    states = initial_states(chans, seed=5, perturb=0.02)
    base = run_gpu(chans, states, nsteps)
    merged = run_gpu(chans, states, nsteps, tuning=dict(merge_classes=merge, graph_steps=8))
    assert base["bad"] == 0 and merged["bad"] == 0
    for key in ("f", "chi", "n", "u", "T", "nw"):
        assert np.array_equal(base[key], merged[key]), key
    ref = run_oracle(chans, states, nsteps, merged["dt"])
    compare(chans, merged, ref, tol=TOL, what=f"launch groups, merge_classes={merge}")


@pytest.mark.parametrize("form", ["fp64", "mixed_f32"])
def test_launch_configurations_bit_identical(form):
    """Class streams (each model class stepping on its own stream), graph
    replay and the identity window mapping give the same bits as the default
    launch configuration; the autotuner's trials advance the state exactly
    like the same number of plain steps."""
    import torch
    h = H()
    chans = _batch_sample(12)
    prec = h.PRECISIONS[form]
    states = initial_states(chans, seed=13, perturb=0.02)
    f0 = torch.from_numpy(np.concatenate([s[0].ravel() for s in states])).cuda()
    c0 = torch.from_numpy(np.concatenate([s[1].ravel() for s in states])).cuda()
    configs = [dict(), dict(class_streams=1), dict(graph_steps=4, class_streams=1, xcd_map=0),
               dict(graph_steps=3, class_streams=0, xcd_map=1)]
    if form == "fp64":   # one launch per stage across the classes (FP64 only)
        configs += [dict(merge_classes=1), dict(merge_classes=2, graph_steps=4),
                    dict(merge_classes=2, xcd_map=0)]
    outs = []
    for cfg in configs:
        s = h.Solver(chans, precision=prec)
        s.set_tuning(**cfg)
        s.set_state(f0, c0)
        s.step(5)
        s.step(6)
        f, c = s.get_state()
        torch.cuda.synchronize()
        outs.append((f.cpu().numpy(), c.cpu().numpy()))
        s.close()
    for k in range(1, len(outs)):
        assert np.array_equal(outs[0][0], outs[k][0]), configs[k]
        assert np.array_equal(outs[0][1], outs[k][1]), configs[k]
    # autotune: direct launches x {one stream, class streams} x 2 mappings and
    # 16-step graphs x 2 mappings, for 2 and (FP64 form) 4 waves per window,
    # (FP64 form) with and without step fusion, and (FP64 form) the launches
    # across classes, (trial + 1) steps each; the four-wave and fused kernels
    # round differently from the two-wave one, so the comparison solver
    # replays the same candidates in the same order
    s = h.Solver(chans, precision=prec)
    s.set_state(f0, c0)
    best = s.autotune(trial_steps=2)
    assert best["ms_per_step"] > 0 and best["graph_steps"] in (0, 16)
    s.step(1)
    f, c = s.get_state()
    r = h.Solver(chans, precision=prec)
    r.set_state(f0, c0)
    fp64 = form == "fp64"
    n_cand = 0
    for sf in ((0, 1) if fp64 else (0,)):
        for wpw in ((2, 4) if fp64 else (2,)):
            for gs in (0, 16):
                for cs in (0, 1):
                    for xm in (1, 0):
                        for mg in (0, 1, 2):
                            if cs and gs > 0:
                                continue
                            if mg and (not fp64 or cs or sf or wpw != 2):
                                continue
                            r.set_tuning(graph_steps=gs, class_streams=cs, xcd_map=xm, waves_per_window=wpw,
                                         step_fusion=sf, merge_classes=mg)
                            r.step(3)
                            n_cand += 1
    assert n_cand == (32 if fp64 else 6)
    r.set_tuning(**{k: best[k] for k in ("graph_steps", "class_streams", "xcd_map", "waves_per_window",
                                         "step_fusion", "merge_classes")})
    r.step(1)
    fr, cr = r.get_state()
    torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy(), fr.cpu().numpy())
    assert np.array_equal(c.cpu().numpy(), cr.cpu().numpy())
    s.close()
    r.close()


@pytest.mark.parametrize("form,tol", [("fp64", 1e-10), ("mixed_f32", 1e-4)])
def test_residual_against_oracle_rhs(form, tol):
    """The residual diagnostic, ||L[y]||_inf / ||y||_inf over f and chi (the
    larger of the two), against the same quantity from the oracle's
    right-hand side on the state the GPU holds."""
    import torch
    import oracle as O
    from gpu_common import to_oracle
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=8, Nx=120, adv=h.WENO5, stretch_A=0.9, T_left=1.0,
                       T_right=2.0, g=-0.5, Kn=kn, dt=-0.5) for kn in (0.01, 1.0)]
    states = initial_states(chans, seed=21, perturb=0.05)
    s = h.Solver(chans, precision=h.PRECISIONS[form])
    s.set_state(torch.from_numpy(np.concatenate([st[0].ravel() for st in states])).cuda(),
                torch.from_numpy(np.concatenate([st[1].ravel() for st in states])).cuda())
    s.step(20)
    f, c = s.get_state()
    nw, mass, bad, res = s.diagnostics(residual=True)
    torch.cuda.synchronize()
    f, c, res = f.cpu().numpy(), c.cpu().numpy(), res.cpu().numpy()
    for k, ch in enumerate(chans):
        fk = s.channel_view(torch.from_numpy(f), k).numpy()
        ck = s.channel_view(torch.from_numpy(c), k).numpy()
        Lf, Lc, _ = O.rhs(to_oracle(ch, dt=oracle_dt(ch)), fk, ck)
        r = max(np.abs(Lf).max() / np.abs(fk).max(), np.abs(Lc).max() / np.abs(ck).max())
        assert abs(res[k] / r - 1) < tol, (form, k, res[k], r)
    s.close()


def test_four_waves_per_window_against_oracle():
    """The four-wave kernel (one wave per momentum half and function) on the
    stretched three-Kn batch, HHLB(15;16) and the edge batch, against the
    oracle (classes without the four-wave kernel keep the two-wave one)."""
    h = H()
    t4 = dict(waves_per_window=4)
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=8, Nx=200, adv=h.WENO5, stretch_A=0.9,
                       T_left=1.0, T_right=2.0, g=-0.5, Kn=kn, dt=-0.5) for kn in (0.01, 0.1, 1.0)]
    _check(chans, 60, perturb=0.05, what="stretched weno5, 4 waves", tuning=t4)
    ch = h.Channel(quad=h.HALF_HERMITE, Q=16, Nx=150, adv=h.WENO5, stretch_A=0.9, T_left=1.0,
                   T_right=1.5, g=-1.0, Kn=0.02, dt=-0.5)
    _check([ch], 25, perturb=0.02, what="HHLB(15;16), 4 waves", tuning=t4)
    edge = [h.Channel(quad=h.HALF_HERMITE, Q=6, N=3, Nx=8, adv=h.WENO5, transverse_dof=2,
                      Kn=math.inf, g=0.3, p0=1.2, T_left=1.2, T_right=0.8, dt=2e-4),
            h.Channel(quad=h.HALF_HERMITE, Q=1, N=0, Nx=59, adv=h.UPWIND3, transverse_dof=2,
                      Kn=0.3, g=-0.2, dt=1e-3),
            h.Channel(quad=h.HALF_HERMITE, Q=4, Nx=117, adv=h.UPWIND3, transverse_dof=0, Kn=0.2,
                      g=-0.2, T_right=1.1, dt=-0.4)]
    _check(edge, 80, perturb=0.03, seed=5, what="edge batch, 4 waves", tuning=t4)


FUSED = dict(step_fusion=1)


def test_step_fusion_small_channel_and_edges():
    """The fused-step kernel (three RK-3 stages per launch, 9-cell halos)
    against the oracle: the small channel (HHLB(3;4), Nx = 64, upwind-3:
    a left-wall window and a right-wall window), Nx = 8 (both walls in one
    window), Q = 1 and 2, no chi, collisionless, positive g, p0 != 1."""
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=4, Nx=64, adv=h.UPWIND3, transverse_dof=2, Kn=0.1,
                       g=-0.1, dt=5e-4),
             h.Channel(quad=h.HALF_HERMITE, Q=6, N=3, Nx=8, adv=h.WENO5, transverse_dof=0,
                       Kn=math.inf, g=0.3, p0=1.2, T_left=1.2, T_right=0.8, dt=2e-4),
             h.Channel(quad=h.HALF_HERMITE, Q=1, N=0, Nx=59, adv=h.UPWIND3, transverse_dof=0,
                       Kn=0.3, g=-0.2, dt=1e-3),
             h.Channel(quad=h.HALF_HERMITE, Q=2, Nx=116, adv=h.WENO5, transverse_dof=2, Kn=0.05,
                       g=-0.7, T_right=1.3, dt=-0.4)]
    _check(chans, 60, perturb=0.03, seed=17, what="fused: small and edge", tuning=FUSED)


def test_step_fusion_window_edges():
    """Channel lengths at the edges of the fused kernel's window rules: one
    window with three (Nx = 8, 58) or two (59, 60) ghosts per wall; 61 (a
    left-wall and a right-wall window); 106 (a remainder of 54 cells after
    the first window, which it avoids); 152 and 428 (interior windows whose
    halo ends next to the right wall's ghosts)."""
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=4, Nx=nx, adv=h.WENO5, transverse_dof=2, Kn=0.08,
                       g=-0.4, T_left=1.0, T_right=1.3, dt=-0.5)
             for nx in (8, 58, 59, 60, 61, 106, 107, 152, 428)]
    _check(chans, 30, perturb=0.03, seed=29, what="fused: window edges", tuning=FUSED)


@pytest.mark.parametrize("Q", [4, 8, 12, 16])
def test_step_fusion_stretched_weno5(Q):
    """Fused steps on stretched WENO-5 channels with unequal walls at three
    Kn (interior windows with 9-cell halos on both sides: Nx = 333 gives a
    left-wall window, six interior ones and a ragged right-wall window),
    from a perturbed start."""
    h = H()
    chans = [h.Channel(quad=h.HALF_HERMITE, Q=Q, Nx=333, adv=h.WENO5, stretch_A=0.9,
                       T_left=1.0, T_right=2.0, g=-0.5, Kn=kn, dt=-0.5) for kn in (0.01, 0.1, 1.0)]
    _check(chans, 30, perturb=0.02, seed=19, what=f"fused: stretched Q={Q}", tuning=FUSED)


def test_step_fusion_batched_sample_with_graphs():
    """The first channels of the batched workload (uneven Nx, Q in {4, 8, 12},
    Kn down to 1e-3) with fused steps under graph replay (two graphs per
    starting copy of the ping-pong pair), against the oracle."""
    chans = _batch_sample(9)
    _check(chans, 25, perturb=0.02, seed=23, what="fused: batched sample, graphs",
           tuning=dict(step_fusion=1, graph_steps=4))
