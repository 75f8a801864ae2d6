"""CPU checks of the C-ABI library: it loads, exports every symbol its header
declares, its host-built tables agree with the oracle's, and argument errors
are reported before any side effect.  No GPU compute is called here."""
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1708_03249_amd as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "hhlb.h")).read()
    names = sorted(set(re.findall(r"\b(hhlb_[a-z_]+)\s*\(", hdr)))
    assert len(names) >= 15
    L = H.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("quad,Q", [(H.HALF_HERMITE, q) for q in (1, 2, 3, 4, 6, 8, 12, 16)] +
                         [(H.FULL_HERMITE, q) for q in (2, 4, 8, 16)] +
                         [(H.HALF_LAGUERRE, q) for q in (1, 2, 3, 4, 6, 8, 12, 16)])
def test_host_tables_match_oracle(quad, Q):
    """The library's tables (recurrence, Jacobi eigenvalues, Christoffel
    weights, force block by integration by parts) against the oracle's
    (monomial coefficients, bisection, Eq. wk_half, Eq. hh_Kk / hh_Kk_L)."""
    p, w = H.nodes(quad, Q)
    K = H.force_matrix(quad, Q)
    po, wo, Ko, *_ = O.tables(quad, Q)
    np.testing.assert_allclose(p, po, rtol=4e-15, atol=0)
    np.testing.assert_allclose(w, wo, rtol=2e-13, atol=0)
    np.testing.assert_allclose(K, Ko, rtol=0, atol=2e-14 * np.abs(Ko).max())


@pytest.mark.parametrize("quad,Q", [(H.HALF_HERMITE, 4), (H.HALF_HERMITE, 8),
                                    (H.HALF_HERMITE, 16), (H.FULL_HERMITE, 16)])
@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.12, 1.7), (-0.3, 0.6), (0.02, 2.6)])
def test_host_equilibrium_matches_oracle(quad, Q, u, T):
    N = Q - 1
    g = H.equilibrium(quad, Q, N, 1.3, u, T)
    go = O.equilibrium(quad, Q, N, 1.3, u, T)
    np.testing.assert_allclose(g, go, rtol=0, atol=2e-15 * np.abs(go).max())


@pytest.mark.parametrize("Q,N", [(4, 3), (8, 7), (8, 4), (16, 15)])
@pytest.mark.parametrize("p0", [1.0, 0.3])
@pytest.mark.parametrize("u,T", [(0.0, 1.0), (0.12, 1.7), (-0.3, 0.6)])
def test_host_equilibrium_laguerre_matches_oracle(Q, N, p0, u, T):
    g = H.equilibrium(H.HALF_LAGUERRE, Q, N, 1.3, u, T, p0)
    go = O.equilibrium(O.LAGUERRE, Q, N, 1.3, u, T, p0)
    np.testing.assert_allclose(g, go, rtol=0, atol=2e-15 * np.abs(go).max())


@pytest.mark.parametrize("Q", [40, 200, 256])
def test_host_half_range_large_q_tables_match_oracle(Q):
    """Half-range HHLB(20;Q) tables of the node-parallel path against the
    oracle (two independent discretised Stieltjes procedures, long double
    and float128), columns of K compared relative to their largest entry."""
    p, w = H.nodes(H.HALF_HERMITE, Q)
    K = H.force_matrix(H.HALF_HERMITE, Q)
    po, wo, Ko, *_ = O.tables(O.HALF, Q)
    np.testing.assert_allclose(p, po, rtol=2e-15, atol=0)
    live = wo > 1e-280
    np.testing.assert_allclose(w[live], wo[live], rtol=1e-13, atol=0)
    assert np.max(np.abs(K - Ko) / np.abs(Ko).max(axis=0)) < 1e-13
    g = H.equilibrium(H.HALF_HERMITE, Q, 20, 1.0, 0.1, 1.2)
    go = O.equilibrium(O.HALF, Q, 20, 1.0, 0.1, 1.2)
    np.testing.assert_allclose(g, go, rtol=0, atol=2e-15 * np.abs(go).max())


@pytest.mark.parametrize("Q", [40, 100, 200])
def test_host_full_range_large_q_tables_match_oracle(Q):
    """Full-range HLB(20;Q) tables of the node-parallel path against the
    oracle (monomial He_l up to Q = 64, its recurrence construction above).
    K's columns span hundreds of decades (the entries of a node's column grow
    like exp(z^2/2) while its populations shrink like exp(-z^2/2)), so each
    column is compared relative to its own largest entry."""
    p, w = H.nodes(H.FULL_HERMITE, Q)
    K = H.force_matrix(H.FULL_HERMITE, Q)
    po, wo, Ko, *_ = O.tables(O.FULL, Q)
    np.testing.assert_allclose(p, po, rtol=4e-15, atol=0)
    live = wo > 1e-280
    np.testing.assert_allclose(w[live], wo[live], rtol=1e-12, atol=0)
    colmax = np.abs(Ko).max(axis=0)
    assert np.max(np.abs(K - Ko) / colmax) < 1e-13
    for u, T in ((0.0, 1.0), (0.15, 1.6), (-0.2, 0.6)):
        g = H.equilibrium(H.FULL_HERMITE, Q, 20, 1.0, u, T)
        go = O.equilibrium(O.FULL, Q, 20, 1.0, u, T)
        np.testing.assert_allclose(g, go, rtol=0, atol=2e-15 * np.abs(go).max())


def test_mixed_forms_reject_laguerre():
    """The mixed-precision forms are built for the half-range Hermite model."""
    ch = H.Channel(quad=H.HALF_LAGUERRE, Q=4, p0=0.4)
    st, h = _create([ch], precision=H.MIXED_F32)
    assert st == -2
    assert "Hermite" in H.lib().hhlb_last_error().decode()
    st, h = _create([ch])
    assert st == 0
    assert H.lib().hhlb_destroy(h) == 0


def test_host_equilibrium_lower_order():
    g = H.equilibrium(H.HALF_HERMITE, 8, 4, 1.0, 0.1, 1.4)
    go = O.equilibrium(O.HALF, 8, 4, 1.0, 0.1, 1.4)
    np.testing.assert_allclose(g, go, rtol=0, atol=2e-15)


def _create(channels, precision=H.FP64):
    import ctypes
    arr = (H._CChannel * len(channels))(*[c._c() for c in channels])
    h = ctypes.c_void_p()
    st = H.lib().hhlb_create(arr, len(channels), precision, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("bad", [
    dict(Q=0), dict(quad=H.FULL_HERMITE, Q=5), dict(N=4, Q=4), dict(Nx=7), dict(adv=3),
    dict(transverse_dof=1), dict(L=0.0), dict(stretch_A=1.0), dict(stretch_A=-0.1),
    dict(Kn=0.0), dict(Kn=-1.0), dict(T_left=0.0), dict(T_right=-1.0), dict(p0=0.0),
    dict(dt=0.0), dict(dt=math.nan), dict(g=math.inf)])
def test_create_rejects_bad_arguments(bad):
    ch = H.Channel(**bad)
    st, h = _create([H.Channel(), ch])
    assert st == -1
    assert "channel 1" in H.lib().hhlb_last_error().decode()


def test_create_unsupported_shape_and_null_calls():
    # Q > 16 runs the node-parallel stage: FP64, N <= 20, half-range Hermite
    # with Q <= 256 or full-range Hermite with Q <= 512
    st, _ = _create([H.Channel(Q=24, N=21)])
    assert st == -2
    st, _ = _create([H.Channel(quad=H.FULL_HERMITE, Q=40, N=21)])
    assert st == -2
    st, _ = _create([H.Channel(quad=H.HALF_LAGUERRE, Q=20)])
    assert st == -2
    st, _ = _create([H.Channel(Q=257)])
    assert st in (-1, -2)
    st, _ = _create([H.Channel(quad=H.FULL_HERMITE, Q=514)])
    assert st in (-1, -2)
    st, _ = _create([H.Channel(quad=H.FULL_HERMITE, Q=21)])
    assert st == -1                              # odd full-range Q
    st, _ = _create([H.Channel(Q=24)], precision=H.MIXED_F32)
    assert st == -2
    # (the largest shapes, half-range Q = 256 and full-range Q = 512, are
    # created by the GPU tests and their tables checked above)
    for ch in (H.Channel(Q=24), H.Channel(quad=H.FULL_HERMITE, Q=20)):
        st, h = _create([ch])
        assert st == 0 and H.lib().hhlb_destroy(h) == 0
    L = H.lib()
    assert L.hhlb_step(None, 1) == -1
    assert L.hhlb_workspace_bytes(None, None) == -1
    st, h = _create([H.Channel()])
    assert st == 0
    assert L.hhlb_step(h, 1) == -6          # no workspace bound yet
    assert L.hhlb_step(h, -1) == -1
    import ctypes
    nb = ctypes.c_size_t()
    assert L.hhlb_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    dts = np.zeros(1)
    assert L.hhlb_time_steps(h, H._dptr(dts)) == 0 and dts[0] == 5e-4
    assert L.hhlb_destroy(h) == 0


def test_cfl_time_step_resolution():
    ch = H.Channel(Q=8, Nx=512, stretch_A=0.9, adv=H.WENO5, Kn=0.01, dt=-0.5)
    st, h = _create([ch])
    assert st == 0
    dts = np.zeros(1)
    assert H.lib().hhlb_time_steps(h, H._dptr(dts)) == 0
    oc = O.Channel(Q=8, Nx=512, A=0.9, Kn=0.01)
    assert dts[0] == pytest.approx(O.cfl_dt(oc, 0.5), rel=1e-12)
    H.lib().hhlb_destroy(h)


def test_precision_argument_and_mixed_workspace():
    """Unknown forms are HHLB_E_ARG; the mixed forms cover the half-range
    model only; their state storage is 4 FP32 copies and 2 16-bit copies per
    function (20 bytes per population against the FP64 form's 24)."""
    import ctypes
    ch = H.Channel(Q=8, Nx=640, Kn=0.1)
    for bad in (-1, 4):
        st, _ = _create([ch], precision=bad)
        assert st == -1
    st, _ = _create([H.Channel(quad=H.FULL_HERMITE, Q=8)], precision=H.MIXED_F32)
    assert st == -2
    sizes = {}
    for prec in (H.FP64, H.MIXED_F32, H.MIXED_BF16, H.MIXED_F16):
        st, h = _create([ch], precision=prec)
        assert st == 0
        nb = ctypes.c_size_t()
        assert H.lib().hhlb_workspace_bytes(h, ctypes.byref(nb)) == 0
        sizes[prec] = nb.value
        H.lib().hhlb_destroy(h)
    pops = 2 * 16 * 640   # f and chi
    assert sizes[H.FP64] - sizes[H.MIXED_F32] == pytest.approx(pops * (24 - 20), abs=4096)
    assert sizes[H.MIXED_F32] == sizes[H.MIXED_BF16] == sizes[H.MIXED_F16]


def test_multi_axes_host_checks():
    """Mixed-quadrature sets (App. A): nodes against the oracle's product set;
    argument and shape errors."""
    from oracle import multi as M
    axes = [H.Axis(H.HALF_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 6, 5),
            H.Axis(H.HALF_LAGUERRE, 3, 2, 0.6)]
    p, w = H.multi_nodes(axes)
    P, W = M.nodes([M.Axis(O.HALF, 4, 3), M.Axis(O.FULL, 6, 5), M.Axis(O.LAGUERRE, 3, 2, 0.6)])
    np.testing.assert_allclose(p, P, rtol=4e-15, atol=0)
    np.testing.assert_allclose(w, W, rtol=2e-13, atol=0)
    import ctypes
    L = H.lib()
    nb = ctypes.c_size_t()
    ax = H._axes(axes)
    assert L.hhlb_multi_workspace_bytes(ax, 3, 1000, ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 1000 * 8 * 6 * 6 * 8
    assert L.hhlb_multi_workspace_bytes(ax, 1, 10, ctypes.byref(nb)) == -1      # d = 1
    assert L.hhlb_multi_workspace_bytes(ax, 4, 10, ctypes.byref(nb)) == -1      # d = 4
    assert L.hhlb_multi_workspace_bytes(ax, 3, -1, ctypes.byref(nb)) == -1
    big = H._axes([H.Axis(H.HALF_HERMITE, 8, 7), H.Axis(H.HALF_HERMITE, 8, 7), H.Axis(H.FULL_HERMITE, 4, 3)])
    assert L.hhlb_multi_workspace_bytes(big, 3, 10, ctypes.byref(nb)) == -2     # V = 1024 > 512
    wide = H._axes([H.Axis(H.HALF_HERMITE, 17, 16), H.Axis(H.FULL_HERMITE, 4, 3)])
    assert L.hhlb_multi_workspace_bytes(wide, 2, 10, ctypes.byref(nb)) == -2    # V_x = 34 > 32
    bad = H._axes([H.Axis(H.HALF_HERMITE, 4, 4), H.Axis(H.FULL_HERMITE, 4, 3)])
    assert L.hhlb_multi_workspace_bytes(bad, 2, 10, ctypes.byref(nb)) == -1     # N >= Q
    odd = H._axes([H.Axis(H.HALF_HERMITE, 4, 3), H.Axis(H.FULL_HERMITE, 5, 3)])
    assert L.hhlb_multi_workspace_bytes(odd, 2, 10, ctypes.byref(nb)) == -1     # odd full-range Q
    F = np.zeros(3)
    assert L.hhlb_multi_step(ax, 3, None, 10, H._dptr(F), 1.0, 1e-3, 1, None, 0, None) == -1
