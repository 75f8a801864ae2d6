"""hhlb_multi_step_noalloc, the entry point for callers that cannot allocate
device memory, through the C ABI against hhlb_multi_step with a caller
workspace (the same kernels and arithmetic, so the results must agree bit
for bit): two calls in a row, the second on fewer points, then a request
beyond the static scratch, which must fail before any side effect."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _state(V, npts, seed):
    # positive, smooth-in-velocity populations: a perturbed constant state
    rng = np.random.default_rng(seed)
    return (1.0 + 0.2 * rng.random((npts, 1))) * (1.0 + 0.1 * rng.random((npts, V))) / V


def test_noalloc_matches_workspace_form():
    import torch
    import paper_1708_03249_amd as H
    axes = [H.Axis(H.HALF_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 4, 3)]
    V = 8 * 4 * 4
    F, Kn, dt = np.array([0.3, -0.2, 0.5]), 0.1, 1e-3
    # first call: 9001 points (ragged against 4 points per block); second: 37
    for npts, nsteps, seed in ((9001, 7, 1), (37, 5, 2)):
        print(f"[noalloc] {npts} points x {nsteps} steps", flush=True)
        f = _state(V, npts, seed)
        ref = torch.from_numpy(f).cuda()
        got = ref.clone()
        s = H.MultiSolver(axes, npts, F, Kn)
        s.step(ref, dt, nsteps)
        H.multi_step_noalloc(axes, got, F, Kn, dt, nsteps)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), (npts, (got - ref).abs().max().item())
        assert not torch.equal(got, torch.from_numpy(f).cuda())   # it did step


def test_noalloc_rejects_too_many_points():
    import torch
    import paper_1708_03249_amd as H
    axes = [H.Axis(H.HALF_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 4, 3)]
    V = 128
    npts = (32 << 20) // (2 * 8 * V) + 1            # beyond the 32 MiB scratch
    f = torch.ones((npts, V), dtype=torch.float64, device="cuda")
    with pytest.raises(H.HHLBError) as e:
        H.multi_step_noalloc(axes, f, [0.1, 0.1, 0.1], 0.1, 1e-3, 1)
    assert e.value.status == -1
    torch.cuda.synchronize()
    assert bool((f == 1.0).all())
