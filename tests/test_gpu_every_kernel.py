"""Every stage-kernel instance the library builds, against the oracle.

One small channel per model shape the kernels are instantiated for -- the
per-half orders Q in {1, 2, 3, 4, 6, 8, 12, 16} (full range: {2, 4, 8, 16}),
f alone (Dt = 0) or f and chi (Dt = 2), WENO-5 or upwind-3 -- all shapes in
one solver, so that each model class runs its own kernel.  The solvers run
4 RK-3 steps from a perturbed equilibrium (Nx = 64..119, so two windows with
a ragged second one; half of the channels on the stretched grid) in every
launch option that selects other kernels: the two-wave stage kernels, the
four-wave ones (f and chi), the fused step, each mixed form, and the
launches across classes (for orders up to 8, 12 and 16, a block per window
or persistent).  FP64 is held to 1e-12 of the oracle, the mixed forms to
1e-5."""
import math
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import compare, initial_states, run_gpu, run_oracle  # noqa: E402

pytestmark = pytest.mark.gpu

HALF_ORDERS = (1, 2, 3, 4, 6, 8, 12, 16)
FULL_ORDERS = (2, 4, 8, 16)
NSTEPS = 4


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _shapes(quad, orders):
    import paper_1708_03249_amd as H
    chans = []
    for Q in orders:
        for dof in (0, 2):
            for adv in (H.WENO5, H.UPWIND3):
                k = len(chans)
                chans.append(H.Channel(quad=quad, Q=Q, Nx=64 + (5 * k) % 56, adv=adv, transverse_dof=dof,
                                       stretch_A=0.6 if k % 2 else 0.0, T_right=1.0 + 0.1 * (k % 5),
                                       g=-0.3 - 0.1 * (k % 4), Kn=0.05 * (1 + k % 3), dt=-0.5))
    return chans


def _run(chans, precision, tuning, tol, what):
    print(f"[every kernel] {what}: {len(chans)} channels, {NSTEPS} steps", flush=True)
    states = initial_states(chans, seed=17, perturb=0.03)
    gpu = run_gpu(chans, states, NSTEPS, precision=precision, tuning=tuning)
    assert gpu["bad"] == 0
    ref = run_oracle(chans, states, NSTEPS, gpu["dt"])
    worst = compare(chans, gpu, ref, tol=tol, what=what)
    print(f"[every kernel] {what}: worst {max(worst.values()):.2e}", flush=True)


@pytest.mark.parametrize("tuning", [None, dict(waves_per_window=4), dict(step_fusion=1)],
                         ids=["two_waves", "four_waves", "fused_step"])
def test_every_half_range_fp64_kernel(tuning):
    import paper_1708_03249_amd as H
    _run(_shapes(H.HALF_HERMITE, HALF_ORDERS), H.FP64, tuning, 1e-12, f"half range FP64 {tuning}")


def test_every_full_range_fp64_kernel():
    import paper_1708_03249_amd as H
    _run(_shapes(H.FULL_HERMITE, FULL_ORDERS), H.FP64, None, 1e-12, "full range FP64")


@pytest.mark.parametrize("form", ["mixed_f32", "mixed_bf16", "mixed_f16"])
def test_every_mixed_kernel(form):
    import paper_1708_03249_amd as H
    _run(_shapes(H.HALF_HERMITE, HALF_ORDERS), H.PRECISIONS[form], None, 1e-5, form)


@pytest.mark.parametrize("merge", [1, 2])
@pytest.mark.parametrize("top", [8, 12, 16])
def test_every_class_group_kernel(top, merge):
    """One launch across classes: the half-range shapes of orders up to
    `top` form four launch groups (f or f and chi, WENO-5 or upwind-3), each
    run by the kernel compiled for orders up to `top`, with a block per window
    (merge 1) or persistent blocks (merge 2), under graph replay."""
    import paper_1708_03249_amd as H
    chans = _shapes(H.HALF_HERMITE, [q for q in HALF_ORDERS if q <= top])
    _run(chans, H.FP64, dict(merge_classes=merge, graph_steps=2), 1e-12,
         f"class groups up to Q = {top}, merge {merge}")
