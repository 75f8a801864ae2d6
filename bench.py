"""Benchmark: velocity-node updates per second of the half-range
Gauss-Hermite lattice Boltzmann time step on one MI355X.

Workload (the largest single-GPU configuration): 256 independent channels,
Nx = 16384 tanh-stretched cells (A = 0.9), HHLB(15;16) (V = 32 momenta),
WENO-5 + TVD RK-3, f and chi (Dt = 2), Kn ~ U[0.005, 0.05] (PCG64 seed 0),
g = -1, T_left = 1, T_right = 1.5, CFL 0.5.  One step = one RK-3 step of
every channel; a node-update is one (x_i, p_k) pair of f and chi advanced
by one step.  Inputs are resident in HBM before the timed region.

Every arithmetic form runs on the same workload, one after the other: the
FP64 form (the primary line) and the mixed forms (FP32 state with a 16-bit
correction word, FP32 advection / collision, force block in FP32, BF16 or
FP16 on the matrix cores, FP64 moments and wall balance).  Each mixed form
reports its speed against the FP64 form and its largest moment difference
from the FP64 form after the same steps (the FP64 form matches the CPU
oracle to 1e-12).

A second workload rides along in the same JSON line ("batched"): 4096
independent channels of uneven Nx, Q, Kn, g and wall-temperature ratio, each
form advancing all of them in one launch per model class and stage, against
the FP64 form stepping each channel as a solver of its own.

Prints one JSON line.  Options: --steps K --warmup W --gpus N (1 only)
--forms fp64,mixed_f32,... --batch-channels C (0 skips the batch)
--no-cpu-baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector

N_CH, NX, Q = 256, 16384, 16


# momentum scale of the half-range Gauss-Laguerre variant.  Its 16 nodes reach
# z = 51.7; at p0 = 0.2 the fastest node sits at 10 thermal speeds and the
# order-15 equilibrium at T = 1 .. 1.5 is positive to rounding, while at
# p0 = 0.1 the truncated Laguerre expansion of the Maxwellian oscillates
# with amplitude 1e4 (see the oracle's equilibrium).
LAGUERRE_P0 = 0.2


def workload(n_ch=N_CH, nx=NX, quad=None):
    """The large workload; quad selects the velocity set (half-range
    Gauss-Hermite by default, or the half-range Gauss-Laguerre one with
    p0 = LAGUERRE_P0)."""
    import paper_1708_03249_amd as H
    from paper_1708_03249_amd.inputs import large_batch_kn
    quad = H.HALF_HERMITE if quad is None else quad
    p0 = LAGUERRE_P0 if quad == H.HALF_LAGUERRE else 1.0
    kns = large_batch_kn(n_ch, seed=0)
    return [H.Channel(quad=quad, Q=Q, N=Q - 1, Nx=nx, adv=H.WENO5, transverse_dof=2,
                      L=1.0, stretch_A=0.9, Kn=kn, g=-1.0, T_left=1.0, T_right=1.5, p0=p0,
                      dt=-0.5) for kn in kns]


def bytes_per_node_update(form="fp64", nfun=2):
    """Algorithmic HBM bytes of one RK-3 step.  One kernel per stage, FP64:
    stage 1 reads y^n and writes y1; stages 2 and 3 read the stage state and
    y^n and write the next state: 8 passes of 8 bytes per function.  Mixed:
    stage 1 reads hi (4) and writes d1 (4); stage 2 reads hi and d1 and writes
    d2; stage 3 reads hi, lo (2) and d2 and writes hi and lo: 36 bytes per
    function.  Fused FP64 step: y^n in, y^{n+1} out, 16 bytes per function
    (the method's minimum)."""
    return nfun * {"fp64": 64, "fp64_fused": 16}.get(form, 36)


def form_precision(H, form):
    """Arithmetic form of a bench form name (fp64_fused: FP64, fused steps)."""
    return H.PRECISIONS["fp64" if form == "fp64_fused" else form]


def form_tuning(form):
    return {"step_fusion": 1} if form == "fp64_fused" else {}


def batch_workload(n_ch=4096, seed=0):
    """The batched workload: n_ch channels drawn from PCG64(seed) (Nx, Q,
    log10 Kn, g, T_right/T_left per channel), uniform grid, WENO-5, f and chi,
    per-channel dt = min(CFL 0.5, Kn/2)."""
    import paper_1708_03249_amd as H
    from paper_1708_03249_amd.inputs import batch_draws
    return [H.Channel(quad=H.HALF_HERMITE, Q=d["Q"], N=d["Q"] - 1, Nx=d["Nx"], adv=H.WENO5,
                      transverse_dof=2, L=1.0, stretch_A=0.0, Kn=d["Kn"], g=d["g"], T_left=1.0,
                      T_right=d["T_right"], p0=1.0, dt=-0.5) for d in batch_draws(n_ch, seed)]


def init_developed(s, torch, np, seed=0, amplitude=0.05):
    """Start state of every timed run: the equilibrium (n, u, T) = (1, 0, 1)
    with each population row of f and chi multiplied by a smooth seeded
    modulation (inputs.smooth_modulation).  A uniform start would leave most
    cells exactly uniform for the first thousands of steps, where the WENO
    smoothness indicators vanish and the degenerate branch runs instead of
    the one a developed flow takes.  Returns the starting mass per channel
    (the modulation moves it off 1 on a stretched grid)."""
    from paper_1708_03249_amd.inputs import smooth_modulation
    s.init_equilibrium(1.0, 0.0, 1.0)
    f, c = s.get_state()
    for k, ch in enumerate(s.channels):
        o0, o1 = int(s.offsets[k]), int(s.offsets[k + 1])
        mf = torch.from_numpy(smooth_modulation(seed + 2 * k, ch.V, ch.Nx, amplitude).ravel())
        f[o0:o1] *= mf.to(f.device)
        if ch.transverse_dof:
            mc = torch.from_numpy(smooth_modulation(seed + 2 * k + 1, ch.V, ch.Nx, amplitude).ravel())
            c[o0:o1] *= mc.to(c.device)
    s.set_state(f, c if s.has_chi else None)
    del f, c
    _, mass0, _ = s.diagnostics()
    return mass0.clone()


TUNING_KEYS = ("graph_steps", "class_streams", "xcd_map", "waves_per_window", "step_fusion", "merge_classes")


def tune_on_sample(H, torch, np, chans, form, trial_steps=10, stride=8):
    """hhlb_autotune on every stride-th channel of the batch (the candidates
    are timed on that sample); returns the chosen configuration."""
    s = H.Solver(chans[::stride], precision=H.PRECISIONS[form])
    init_developed(s, torch, np)
    best = s.autotune(trial_steps=trial_steps)
    torch.cuda.synchronize()
    s.close()
    torch.cuda.empty_cache()
    return best


def run_batch(H, torch, np, args):
    """Batched workload: every form advances all channels in one launch per
    class and stage (or per class and step with step fusion); compared with
    the FP64 form stepping each channel as its own solver (timed on a
    sample of channels).  Legs: each form in the default launch
    configuration (direct launches, classes in turn on one stream); the FP64
    form with fused steps; the FP64 form with one launch per stage across
    its classes (a block per window, and persistent blocks), replayed as
    16-step HIP graphs; and each form in the configuration hhlb_autotune
    picks on every 8th channel, replayed as HIP graphs when it chooses them."""
    chans = batch_workload(args.batch_channels)
    nu_step = sum(c.V * c.Nx for c in chans)
    out = {"workload": f"{len(chans)} channels, Nx~U{{64..1024}}, Q~U{{4,8,12}}, log10 Kn~U[-3,1], "
                       "g~U[-1,0], T_right/T_left~U[1,2] (PCG64 seed 0), uniform grid, WENO5+RK3, "
                       "f and chi, dt=min(CFL 0.5, Kn/2), smoothly modulated start",
           "node_updates_per_step": nu_step, "steps": args.batch_steps, "forms": {}}
    legs = [("fp64", "fp64", {}), ("fp64_fused", "fp64", {"step_fusion": 1}),
            ("fp64_one_launch", "fp64", {"merge_classes": 1, "graph_steps": 16}),
            ("fp64_persistent", "fp64", {"merge_classes": 2, "graph_steps": 16}),
            ("mixed_f32", "mixed_f32", {})]
    if not args.no_batch_tune:
        for form in ("fp64", "mixed_f32"):
            print(f"[bench] batch {form}: autotune on every 8th channel", file=sys.stderr, flush=True)
            best = tune_on_sample(H, torch, np, chans, form)
            legs.append((f"{form}_tuned", form, {k: best[k] for k in TUNING_KEYS}))
    ref = None
    for name, form, tuning in legs:
        s = H.Solver(chans, precision=H.PRECISIONS[form])
        if tuning:
            s.set_tuning(**tuning)
        mass0 = init_developed(s, torch, np)
        print(f"[bench] batch {name}: {len(chans)} channels, {args.batch_steps} steps",
              file=sys.stderr, flush=True)
        used = s.tuning()
        s.step(args.warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(args.batch_steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        nw, mass, bad = s.diagnostics()
        mom = s.moments()
        torch.cuda.synchronize()
        assert int(bad.item()) == 0, f"batch {name}: non-finite populations"
        used.pop("ms_per_step", None)
        # algorithmic HBM bytes of a step over its time (every class together)
        bform = "fp64_fused" if tuning.get("step_fusion") else form
        gbs = bytes_per_node_update(bform) * nu_step / (ms / args.batch_steps / 1e3) / 1e9
        rec = {"value": nu_step * args.batch_steps / (ms / 1e3), "unit": "node-updates/s",
               "ms_per_step": ms / args.batch_steps, "tuning": used,
               "launches_per_stage": s.launch_info()[0],
               "hbm": {"algorithmic_bytes_per_node_update": bytes_per_node_update(bform),
                       "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)},
               "mass_drift": float(((mass - mass0) / mass0).abs().max().item())}
        if name == "fp64":
            ref = mom
        else:
            rec["err_vs_fp64"] = moment_diff(np, ref, mom)
        out["forms"][name] = rec
        s.close()
        del mom
        torch.cuda.empty_cache()
    # per-instance FP64: one solver (and its own launches) per channel, on an
    # evenly spaced sample of the channels
    sample = chans[::max(1, len(chans) // args.instance_sample)][:args.instance_sample]
    print(f"[bench] per-instance fp64: {len(sample)} solvers x {args.instance_steps} steps",
          file=sys.stderr, flush=True)
    solvers = []
    for c in sample:
        s = H.Solver([c])
        init_developed(s, torch, np)
        s.step(1)
        solvers.append(s)
    torch.cuda.synchronize()
    steps = args.instance_steps
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nu = sum(c.V * c.Nx for c in sample) * steps
    for s in solvers:
        s.close()
    out["per_instance_fp64"] = {"value": nu / el, "unit": "node-updates/s",
                                "sample": f"{len(sample)} of the channels, one solver each, "
                                          f"{steps} steps each, launched one after another"}
    out["batched_vs_per_instance"] = {f: round(r["value"] / out["per_instance_fp64"]["value"], 1)
                                      for f, r in out["forms"].items()}
    out["vs_fp64_batched"] = {f: round(r["value"] / out["forms"]["fp64"]["value"], 3)
                              for f, r in out["forms"].items() if f != "fp64"}
    return out


def steady_workload():
    """The steady-state study: HHLB(7;8) and the full-range HLB(15;16), both
    V = 16, on Nx = 512 cells stretched towards the walls (A = 0.9), WENO-5,
    T_left = 1, T_right = 2, g = -0.5, Kn in {0.01, 0.1, 1}, CFL 0.5."""
    import paper_1708_03249_amd as H
    return [H.Channel(quad=quad, Q=Q, N=Q - 1, Nx=512, adv=H.WENO5, transverse_dof=2, L=1.0,
                      stretch_A=0.9, Kn=kn, g=-0.5, T_left=1.0, T_right=2.0, p0=1.0, dt=-0.5)
            for quad, Q in ((H.HALF_HERMITE, 8), (H.FULL_HERMITE, 16)) for kn in (0.01, 0.1, 1.0)]


def run_steady(H, torch, np, args):
    """Advance the steady-state study (all six channels in one solver) until
    every channel's residual is below args.residual (checked every
    args.check_every steps), reporting the steps taken and the steady flow."""
    chans = steady_workload()
    s = H.Solver(chans)
    s.init_equilibrium(1.0, 0.0, 1.0)
    done, t0, res = 0, time.perf_counter(), None
    conv = [None] * len(chans)
    while done < args.max_steps:
        s.step(args.check_every)
        done += args.check_every
        _, _, bad, r = s.diagnostics(residual=True)
        r = r.cpu().numpy()
        if int(bad.item()):
            raise RuntimeError("steady study: non-finite populations")
        for k in range(len(chans)):
            if conv[k] is None and r[k] <= args.residual:
                conv[k] = done
        if done % (20 * args.check_every) == 0:
            print(f"[steady] {done} steps, residuals {' '.join(f'{x:.1e}' for x in r)}",
                  file=sys.stderr, flush=True)
        res = r
        if all(c is not None for c in conv):
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n, u, T = (x.cpu().numpy() for x in s.moments())
    nw, mass, _ = s.diagnostics()
    nw, mass = nw.cpu().numpy(), mass.cpu().numpy()
    rows = []
    for k, ch in enumerate(chans):
        a, b = s.cells[k], s.cells[k + 1]
        rows.append({"model": ("HHLB" if ch.quad == H.HALF_HERMITE else "HLB") + f"({ch.N};{ch.Q})",
                     "Kn": ch.Kn, "steps_to_residual": conv[k], "residual": float(res[k]),
                     "dt": float(s.dt[k]), "max_abs_u": float(np.abs(u[a:b]).max()),
                     "n_left": float(n[a]), "n_right": float(n[b - 1]),
                     "T_left_cell": float(T[a]), "T_right_cell": float(T[b - 1]),
                     "n_wall": [float(x) for x in nw[k]], "mass": float(mass[k])})
    s.close()
    return {"workload": steady_workload.__doc__.split("\n\n")[0].replace("\n", " ").strip(),
            "residual_target": args.residual, "steps": done, "wall_s": round(wall, 1), "channels": rows}


def flops_per_node_update(Q=Q, N=Q - 1, nfun=2, nc=8):
    """Floating-point operations of one node-update (both functions, three
    stages) as the FP64 stage kernel executes them, counting an FMA as two:
    per node and function, the lane-parallel WENO-5 face value (smoothness
    indicators, candidates and weights of the triple decomposition: 58), flux
    difference and RK combination (6), structured force matrix (half block
    plus rank-1 term: 2(Q+2)) and BGK (4); per cell and shared by its 2Q
    nodes, the moment sums (7 per node) and the equilibrium: the M = (N+2)//2
    main points and nc correction points of each half, N+1 recurrence levels
    of 8 flops each, then the table contraction 2Q (N+1) x 2."""
    V = 2 * Q
    M = (N + 2) // 2
    per_node_fn = 58 + 6 + 2 * (Q + 2) + 4
    per_cell = 7 * V + 2 * (M + nc) * (N + 1) * 8 + V * (N + 1) * 2
    return 3 * (nfun * per_node_fn + per_cell / V)


def ladder_points(counts, reach, y):
    """Correction points per half that the equilibrium's ladder (counts,
    reach from hhlb_equilibrium_ladder) selects for a wave whose largest
    |y0| = |u| sqrt(m/T) is y: the smallest count whose calibrated reach
    covers y; beyond the top count's reach, the top count on the smallest
    power-of-two number of panels (at most 64) that covers it."""
    if y <= 0:
        return 0
    for n, r in zip(counts[1:], reach[1:]):
        if r >= y:
            return n
    if not reach[-1] > 0:
        return counts[-1]
    P = 2
    while P < 64 and reach[-1] * P < y:
        P *= 2
    return counts[-1] * P


def mean_ladder_points(s, mom, np):
    """Average correction points per half over the windows of 58 cells, from
    the final moments: each window takes the ladder count covering its
    largest |u|/sqrt(T)."""
    n, u, T = mom
    y = (u.abs() / T.clamp_min(1e-300).sqrt()).cpu().numpy()
    counts, reach = s.equilibrium_ladder(0)
    tot, nw = 0.0, 0
    for k, ch in enumerate(s.channels):
        a, b = int(s.cells[k]), int(s.cells[k + 1])
        for i0 in range(a, b, 58):
            tot += ladder_points(counts, reach, float(y[max(a, i0 - 3):min(b, i0 + 61)].max()))
            nw += 1
    return tot / max(nw, 1)


def measured_counter(form, key):
    """A figure (e.g. the MFMA busy fraction) from the committed rocprofv3
    counter record of the stage kernel, if it was taken on the kernel source
    built now; else None."""
    rec = _profile_record(form)
    return None if rec is None else rec.get(key)


def _profile_record(form="fp64", name=None):
    import hashlib
    if name is None:
        name = "stage_kernel_traffic.json" if form == "fp64" else f"stage_kernel_{form}_traffic.json"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for f in rec.get("kernel_source_files", ()):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("kernel_source_sha256"):
        return None
    return rec


def measured_traffic(form="fp64", name=None):
    """HBM bytes per stage launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes, if they were taken on the kernel source (the kernel's
    sources and the build flags) built now.  `name` picks another record."""
    rec = _profile_record(form, name)
    if rec is None:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def cpu_baseline(H, torch, np, forms, steps, n_parity=4, max_threads=16):
    """Time the plain CPU oracle on a bounded sample of the same workload and
    check every GPU form against it on the same start.

    The sample: `steps` RK-3 steps of channel 0 on one core, then of the
    first C channels on C threads, one channel each, C the cores this process
    may run on (sched_getaffinity), capped at max_threads (the host share of
    one GPU).  Start: the oracle's equilibrium (1, 0, 1) times the smooth
    modulation of the timed runs (the seeds of init_developed), and the
    oracle's own CFL time step.  Each form then advances the first n_parity
    channels from that same start on the GPU, and its moments are compared
    with the oracle's after the same steps."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle as O
    from paper_1708_03249_amd.inputs import smooth_modulation
    affinity = len(os.sched_getaffinity(0))
    threads = max(1, min(affinity, max_threads))
    chans = workload()[:max(threads, n_parity)]
    V = 2 * Q

    def ochan(ch):
        oc = O.Channel(quad=O.HALF, Q=Q, N=Q - 1, Nx=NX, adv=O.WENO5, Dt=2, A=0.9, Kn=ch.Kn,
                       g=-1.0, T_left=1.0, T_right=1.5)
        oc.dt = O.cfl_dt(oc, 0.5)
        return oc

    def start(c):
        oc = ochan(chans[c])
        f, chi = O.initial_state(oc)
        return oc, f * smooth_modulation(2 * c, V, NX, 0.05), chi * smooth_modulation(2 * c + 1, V, NX, 0.05)

    def one(c):
        oc, f, chi = start(c)
        f, chi, _ = O.run(oc, steps, f, chi)
        return O.moments(oc, f, chi)

    O.lib()
    t0 = time.perf_counter()
    one(0)
    el1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        ref = list(ex.map(one, range(threads)))
    eln = time.perf_counter() - t0
    nu_ch = NX * V * steps
    out = {"value": threads * nu_ch / eln, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{threads} of the 256 channels (Nx={NX}, HHLB(15;16), f and chi) on {threads} "
                     f"threads, one channel each, {steps} RK-3 steps from the timed runs' start, "
                     f"{eln:.1f} s",
           "cores_available": affinity,
           "one_core": {"value": nu_ch / el1, "unit": "node-updates/s", "cores": 1,
                        "sample": f"channel 0, {steps} RK-3 steps, {el1:.1f} s"}}
    # every GPU form against the oracle on the first n_parity channels
    starts = [start(c) for c in range(n_parity)]
    errs = {}
    for form in forms:
        s = H.Solver(chans[:n_parity], precision=form_precision(H, form))
        s.set_tuning(**form_tuning(form))
        for k, (oc, _, _) in enumerate(starts):
            assert abs(s.dt[k] - oc.dt) <= 4.5e-16 * oc.dt, (form, k, s.dt[k], oc.dt)
        f = torch.from_numpy(np.concatenate([st[1].ravel() for st in starts])).cuda()
        c = torch.from_numpy(np.concatenate([st[2].ravel() for st in starts])).cuda()
        s.set_state(f, c)
        del f, c
        s.step(steps)
        n, u, T = (x.cpu().numpy() for x in s.moments())
        s.close()
        e = {"err_n": 0.0, "err_u": 0.0, "err_T": 0.0}
        for k in range(n_parity):
            rn, ru, rT = ref[k]
            a, b = k * NX, (k + 1) * NX
            e["err_n"] = max(e["err_n"], float(np.abs(n[a:b] - rn).max() / np.abs(rn).max()))
            e["err_u"] = max(e["err_u"], float(np.abs(u[a:b] - ru).max()))
            e["err_T"] = max(e["err_T"], float(np.abs(T[a:b] - rT).max() / np.abs(rT).max()))
        errs[form] = e
        torch.cuda.empty_cache()
    out["err_vs_oracle"] = {"channels": n_parity, "steps": steps, "start": "the timed runs' start "
                            "(equilibrium (1, 0, 1) times the seeded smooth modulation)", "forms": errs}
    return out


def copy_bandwidth(torch, mib=1024, reps=5):
    """Bandwidth a plain device copy of mib MiB reaches on this GPU (read +
    write bytes over the copy time, best of reps): the practical ceiling the
    stage kernels' HBM fraction is also quoted against."""
    n = mib * 2**20 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / (best / 1e3) / 1e9


def run_form(H, torch, np, chans, form, args):
    """Warm up, time args.steps steps of one arithmetic form; return its
    record and the final moments (device tensors)."""
    s = H.Solver(chans, precision=form_precision(H, form))
    s.set_tuning(waves_per_window=args.waves_per_window, **form_tuning(form))
    mass0 = init_developed(s, torch, np)
    print(f"[bench] {form}: {len(chans)} channels x Nx={NX}, V={2 * Q}; workspace "
          f"{s.ws_bytes / 2**30:.2f} GiB; warmup {args.warmup}", file=sys.stderr, flush=True)
    s.step(args.warmup)
    torch.cuda.synchronize()
    launches, windows = s.launch_info()
    stream = s.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    nw, mass, bad = s.diagnostics()
    mom = s.moments()
    torch.cuda.synchronize()
    assert int(bad.item()) == 0, f"{form}: non-finite populations"
    mass_err = float(((mass - mass0) / mass0).abs().max().item())   # relative, from the start
    node_updates = sum(c.V * c.Nx for c in chans) * args.steps
    value = node_updates / (ms / 1e3)
    # dominant kernel: the stage kernel (every launch of the timed region),
    # or the fused-step kernel (one launch per class and step)
    per_step = 1 if form == "fp64_fused" else 3
    n_launch = per_step * args.steps * launches
    avg_launch_s = ms / 1e3 / n_launch
    nu_per_launch = sum(c.V * c.Nx for c in chans) / launches
    bpl = bytes_per_node_update(form) / per_step * nu_per_launch
    nc = mean_ladder_points(s, mom, np)
    # the fused kernel also computes its halo lanes: 64 lanes per 46 outputs
    redundancy = 64.0 / 46.0 if form == "fp64_fused" else 1.0
    fpl = flops_per_node_update(nc=nc) * redundancy / per_step * nu_per_launch
    gbs = bpl / avg_launch_s / 1e9
    tfs = fpl / avg_launch_s / 1e12
    # the scope's roof for this streaming stencil is HBM (128 B per
    # node-update in FP64, 72 in the mixed forms); the vector-ALU fraction of
    # the executed flop count rides along
    kname = {"fp64": "hhlb::stage_kernel_half<16,2,0> (one RK-3 stage, FP64)",
             "fp64_fused": "hhlb::fused_kernel_half<16,2,0> (one whole RK-3 step, FP64)"}.get(
        form, f"hhlb::stage_kernel_mixed<16,2,0,{form_precision(H, form)}> (one RK-3 stage, {form})")
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(form),
            "kernel": kname, "algorithmic_bytes_per_node_update": bytes_per_node_update(form),
            "algorithmic_bytes_per_launch": bpl,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "alu": {"flops_per_node_update": round(flops_per_node_update(nc=nc) * redundancy, 1),
                    "correction_points_per_half": round(nc, 2),
                    "achieved_tflops": round(tfs, 2), "peak_tflops": FP64_VECTOR_PEAK_TFLOPS,
                    "frac": round(tfs / FP64_VECTOR_PEAK_TFLOPS, 4)},
            "mfma_busy": measured_counter(form, "mfma_busy_frac")}
    rec = {"value": value, "ms_per_step": ms / args.steps, "roofline": roof, "mass_drift": mass_err,
           "wall_s": round(wall, 3), "node_updates_per_step": node_updates // args.steps}
    s.close()
    return rec, mom


def run_ballistic(H, torch, np, nx=24, steps=2000, warmup=32):
    """The node-parallel path on the paper's ballistic set-up (Sec. V.E):
    HHLB(20;200), V = 400, Nx = 24 (or nx), A = 0.99, dt = 1e-4, Kn = inf, no
    chi, its eight cases (g_p in {0.1, 1} x Delta T in {0.6, 0.3, 0, -0.4})
    as one batch, from the equilibrium at rest.  The paper's dt = 1e-4 is
    stable at Nx = 24 only (the stretched grid's smallest cell shrinks with
    Nx); other nx take the CFL 0.5 step.  HIP events on the solver's
    stream."""
    dt = 1e-4 if nx == 24 else -0.5
    cases = [(gp, dT) for gp in (0.1, 1.0) for dT in (0.6, 0.3, 0.0, -0.4)]
    chans = [H.Channel(quad=H.HALF_HERMITE, Q=200, N=20, Nx=nx, adv=H.WENO5, transverse_dof=0,
                       stretch_A=0.99, Kn=math.inf, g=-gp, T_left=1 - dT, T_right=1 + dT, dt=dt)
             for gp, dT in cases]
    s = H.Solver(chans)
    s.init_equilibrium()
    s.step(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, _, bad = s.diagnostics()
    assert int(bad.item()) == 0, "ballistic: non-finite populations"
    nu = sum(c.V * c.Nx for c in chans)
    s.close()
    return {"workload": f"HHLB(20;200) V=400, 8 channels (the paper's ballistic cases) x Nx={nx} "
                        "tanh-stretched (A=0.99), WENO5+RK3, Kn=inf, "
                        + ("dt=1e-4" if nx == 24 else "CFL 0.5") + ", f only, FP64, "
                        "node-parallel stage (cell kernel + MFMA node kernel per RK stage)",
            "value": nu * steps / (ms / 1e3), "unit": "node-updates/s",
            "ms_per_step": ms / steps, "steps": steps}


def run_small(H, torch, np, steps=20000, warmup=64):
    """The small channel of the parity tests, HHLB(3;4), Nx = 64, third-order
    upwind, f and chi, Kn = 0.1, g = -0.1, equal walls, dt = 5e-4, from the
    equilibrium: 20 000 steps (t = 10) as 64-step HIP graphs, per-stage
    launches and fused steps.  One channel of two windows is launch-bound:
    this is the latency of a step.  HIP events on the solver's stream."""
    ch = H.Channel(quad=H.HALF_HERMITE, Q=4, N=3, Nx=64, adv=H.UPWIND3, transverse_dof=2, Kn=0.1,
                   g=-0.1, dt=5e-4)
    rec = {"workload": "HHLB(3;4) V=8, one channel, Nx=64 uniform, upwind-3+RK3, f and chi, Kn=0.1, "
                       "g=-0.1, equal walls, dt=5e-4, 64-step HIP graphs", "steps": steps}
    for name, fusion in (("per_stage", 0), ("fused", 1)):
        s = H.Solver([ch])
        s.set_tuning(graph_steps=64, step_fusion=fusion)
        s.init_equilibrium()
        s.step(warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s.stream)
        s.step(steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        _, _, bad = s.diagnostics()
        assert int(bad.item()) == 0, "small channel: non-finite populations"
        s.close()
        rec[name] = {"value": ch.V * ch.Nx * steps / (ms / 1e3), "unit": "node-updates/s",
                     "us_per_step": 1e3 * ms / steps}
    return rec


def run_multi(H, torch, np, npts=1_000_000, steps=10, warmup=2):
    """The mixed-quadrature velocity space of App. A (homogeneous gas): a
    3-D product set HH(4) x H(4) x H(4) (V = 8 x 4 x 4 = 128, N = 3 per
    axis), npts points started at the discrete Maxwellian w_v modulated by a
    seeded smooth factor, F = (0.3, -0.2, 0.5), Kn = 0.1, dt = 1e-3.  HIP
    events on the stream the steps run on.  Algorithmic HBM bytes per
    node-update per RK-3 step: 64 (reads of y_s and y^n, writes of the next
    stage; 8-byte values)."""
    axes = [H.Axis(H.HALF_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 4, 3)]
    p, w = H.multi_nodes(axes)
    V = w.size
    rng = np.random.default_rng(0)
    mod = 1.0 + 0.05 * np.sin(rng.random((npts, 1)) * 2 * np.pi + np.arange(V)[None, :] * 0.1)
    f = torch.from_numpy(w[None, :] * mod).cuda()
    del mod
    s = H.MultiSolver(axes, npts, [0.3, -0.2, 0.5], 0.1)
    s.step(f, 1e-3, warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(f, 1e-3, steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    assert bool(torch.isfinite(f).all()), "multi: non-finite populations"
    nu = npts * V
    gbs = 64.0 * nu / (ms / 1e3) / 1e9
    out = {"workload": f"App. A mixed quadrature, homogeneous gas: HH(4) x H(4) x H(4) (V = {V}, N = 3 per "
                       f"axis), {npts} points, F = (0.3, -0.2, 0.5), Kn = 0.1, dt = 1e-3, FP64",
           "value": nu / (ms / 1e3), "unit": "node-updates/s", "ms_per_step": ms, "steps": steps,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(name="multi_kernel_traffic.json"),
                        "kernel": "hhlb::multi_kernel (one RK-3 stage)",
                        "algorithmic_bytes_per_node_update_per_step": 64,
                        "algorithmic_bytes_per_launch": 64.0 * nu / 3,
                        "traffic_unit": "HBM bytes per launch, average over the three stages "
                                        "(rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)"}}
    del f
    torch.cuda.empty_cache()
    return out


def moment_diff(np, a, b):
    """err_n = max|dn|/max n, err_u = max|du|/sqrt(T_left), err_T = max|dT|/max T."""
    n0, u0, T0 = a
    n1, u1, T1 = b
    return {"err_n": ((n1 - n0).abs().max() / n0.abs().max()).item(),
            "err_u": (u1 - u0).abs().max().item(),
            "err_T": ((T1 - T0).abs().max() / T0.abs().max()).item()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp64,mixed_f32,mixed_bf16,mixed_f16,fp64_fused",
                    help="arithmetic forms to time; the first is the primary line")
    ap.add_argument("--waves-per-window", type=int, default=2, choices=(2, 4),
                    help="stage-kernel shape for the large workload (4: FP64 four-wave kernel)")
    ap.add_argument("--batch-channels", type=int, default=4096,
                    help="channels of the batched uneven workload (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--no-batch-tune", action="store_true",
                    help="skip the autotuned legs of the batched workload")
    ap.add_argument("--instance-sample", type=int, default=64)
    ap.add_argument("--instance-steps", type=int, default=20)
    ap.add_argument("--steady", action="store_true",
                    help="only run the steady-state study to --residual")
    ap.add_argument("--residual", type=float, default=1e-10)
    ap.add_argument("--check-every", type=int, default=1000)
    ap.add_argument("--max-steps", type=int, default=3_000_000)
    ap.add_argument("--no-ballistic", action="store_true",
                    help="skip the HHLB(20;200) ballistic record (the node-parallel path)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small-channel latency record (HHLB(3;4), Nx=64)")
    ap.add_argument("--no-multi", action="store_true",
                    help="skip the mixed-quadrature (App. A) record")
    ap.add_argument("--multi-only", action="store_true",
                    help="only run the mixed-quadrature (App. A) record")
    ap.add_argument("--ballistic-only", action="store_true",
                    help="only run the HHLB(20;200) ballistic record")
    ap.add_argument("--ballistic-nx", type=int, default=24,
                    help="cells per channel of the ballistic record")
    ap.add_argument("--ballistic-steps", type=int, default=2000)
    ap.add_argument("--no-laguerre", action="store_true",
                    help="skip the FP64 timing of the half-range Gauss-Laguerre velocity set")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe_mib:
        import torch
        n = args.copy_probe_mib * 2**20 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 8, "copies": 3}))
        return
    if args.multi_only:
        import numpy as np
        import torch
        import paper_1708_03249_amd as H
        print(json.dumps({"multi_d": run_multi(H, torch, np)}), flush=True)
        return
    if args.ballistic_only:
        import numpy as np
        import torch
        import paper_1708_03249_amd as H
        print(json.dumps({"ballistic_q200": run_ballistic(H, torch, np, nx=args.ballistic_nx,
                                                          steps=args.ballistic_steps)}), flush=True)
        return
    if args.steady:
        import numpy as np
        import torch
        import paper_1708_03249_amd as H
        print(json.dumps({"steady": run_steady(H, torch, np, args)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "channels are independent and would shard across GPUs without exchange, "
              "which is not built here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1708_03249_amd as H

    chans = workload()
    forms = [f for f in args.forms.split(",") if f]
    results, ref_moments = {}, None
    for form in forms:
        r, mom = run_form(H, torch, np, chans, form, args)
        if form == "fp64":
            ref_moments = mom
        elif ref_moments is not None:
            r["err_vs_fp64"] = {k: float(v) for k, v in moment_diff(np, ref_moments, mom).items()}
        results[form] = r
        del mom
        torch.cuda.empty_cache()
    prim = results[forms[0]]
    copy_gbs = copy_bandwidth(torch)
    for r in results.values():
        r["roofline"]["copy_GBps"] = round(copy_gbs, 1)
        r["roofline"]["frac_of_copy"] = round(r["roofline"]["achieved"] / copy_gbs, 4)
    out = {
        "metric": "velocity-node updates/s (x·p_x)",
        "value": prim["value"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if forms[0] == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{len(chans)} channels x Nx={NX} tanh-stretched (A=0.9), "
                               "HHLB(15;16) V=32, WENO5+RK3, f and chi, Kn~U[0.005,0.05], g=-1, "
                               "T_right/T_left=1.5, CFL 0.5, start: equilibrium (1, 0, 1) times a smooth "
                               "seeded modulation (amplitude 0.05) of every population row",
                   "channels": len(chans), "Nx": NX, "V": 2 * Q, "form": forms[0],
                   "node_updates_per_step": prim["node_updates_per_step"]},
        "roofline": prim["roofline"],
        "mass_drift": prim["mass_drift"],
        "forms": {f: {k: v for k, v in r.items() if k != "roofline"} | {"roofline": r["roofline"]}
                  for f, r in results.items() if f != forms[0]},
    }
    if "fp64" in results:
        out["speed_vs_fp64"] = {f: round(r["value"] / results["fp64"]["value"], 3)
                                for f, r in results.items() if f != "fp64"}
    if not args.no_laguerre:
        # the same kernels with the half-range Gauss-Laguerre tables (FP64)
        lag = workload(quad=H.HALF_LAGUERRE)
        r, mom = run_form(H, torch, np, lag, "fp64", args)
        del mom
        torch.cuda.empty_cache()
        out["half_range_laguerre"] = {
            "workload": f"the large workload with the half-range Gauss-Laguerre velocity set "
                        f"(Q=16, V=32, p0={LAGUERRE_P0}), FP64",
            "value": r["value"], "unit": "node-updates/s", "ms_per_step": r["ms_per_step"],
            "mass_drift": r["mass_drift"], "avg_launch_us": r["roofline"]["avg_launch_us"]}
    if not args.no_small:
        print("[bench] small channel HHLB(3;4), Nx=64: 20000 steps", file=sys.stderr, flush=True)
        out["small_channel"] = run_small(H, torch, np)
    if not args.no_ballistic:
        print("[bench] ballistic HHLB(20;200): 8 channels x Nx=24", file=sys.stderr, flush=True)
        out["ballistic_q200"] = run_ballistic(H, torch, np, nx=args.ballistic_nx,
                                              steps=args.ballistic_steps)
    if not args.no_multi:
        print("[bench] mixed quadrature (App. A): 1e6 points x V=128", file=sys.stderr, flush=True)
        out["multi_d"] = run_multi(H, torch, np)
    if args.batch_channels > 0:
        out["batched"] = run_batch(H, torch, np, args)
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline and oracle parity: {args.cpu_steps} steps",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(H, torch, np, forms, args.cpu_steps)
        out["err_vs_oracle"] = out["cpu_baseline"].pop("err_vs_oracle")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
