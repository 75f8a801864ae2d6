"""Python binding of libhhlb.so, the gfx950 library for the time step of the
half-range Gauss-Hermite lattice Boltzmann model with a force term
(arXiv:1708.03249).

Argument marshalling only: every arithmetic step of the time step runs in the
HIP kernels behind ``include/hhlb.h``.  PyTorch provides device memory and
the stream.  The library must be built (``python -m paper_1708_03249_amd.build``);
importing this module fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HHLB_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("HHLB_LIBRARY") or os.path.join(_HERE, "libhhlb.so")

HALF_HERMITE, FULL_HERMITE, HALF_LAGUERRE = 0, 1, 2
WENO5, UPWIND3 = 0, 1
FP64, MIXED_F32, MIXED_BF16, MIXED_F16 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "mixed_f32": MIXED_F32, "mixed_bf16": MIXED_BF16, "mixed_f16": MIXED_F16}

_STATUS = {0: "HHLB_OK", -1: "HHLB_E_ARG", -2: "HHLB_E_UNSUPPORTED", -3: "HHLB_E_HIP",
           -4: "HHLB_E_NOMEM", -5: "HHLB_E_NUMERIC", -6: "HHLB_E_STATE"}


class HHLBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _CTuning(ctypes.Structure):
    _fields_ = [("graph_steps", ctypes.c_int32), ("class_streams", ctypes.c_int32),
                ("xcd_map", ctypes.c_int32), ("waves_per_window", ctypes.c_int32),
                ("step_fusion", ctypes.c_int32), ("merge_classes", ctypes.c_int32),
                ("ms_per_step", ctypes.c_float)]

    def as_dict(self):
        return {"graph_steps": self.graph_steps, "class_streams": self.class_streams,
                "xcd_map": self.xcd_map, "waves_per_window": self.waves_per_window,
                "step_fusion": self.step_fusion, "merge_classes": self.merge_classes,
                "ms_per_step": self.ms_per_step}


class _CChannel(ctypes.Structure):
    _fields_ = [("quad", ctypes.c_int32), ("Q", ctypes.c_int32), ("N", ctypes.c_int32),
                ("Nx", ctypes.c_int32), ("adv", ctypes.c_int32),
                ("transverse_dof", ctypes.c_int32), ("L", ctypes.c_double),
                ("stretch_A", ctypes.c_double), ("Kn", ctypes.c_double), ("g", ctypes.c_double),
                ("T_left", ctypes.c_double), ("T_right", ctypes.c_double),
                ("p0", ctypes.c_double), ("dt", ctypes.c_double)]


@dataclass
class Channel:
    """A force-driven channel between diffuse walls (see include/hhlb.h)."""
    quad: int = HALF_HERMITE
    Q: int = 4
    N: int = -1
    Nx: int = 64
    adv: int = WENO5
    transverse_dof: int = 2
    L: float = 1.0
    stretch_A: float = 0.0
    Kn: float = 0.1
    g: float = -0.1
    T_left: float = 1.0
    T_right: float = 1.0
    p0: float = 1.0
    dt: float = 5e-4

    @property
    def V(self) -> int:
        return self.Q if self.quad == FULL_HERMITE else 2 * self.Q

    def _c(self) -> _CChannel:
        return _CChannel(self.quad, self.Q, self.N, self.Nx, self.adv, self.transverse_dof,
                         self.L, self.stretch_A, self.Kn, self.g, self.T_left, self.T_right,
                         self.p0, self.dt)


class _CAxis(ctypes.Structure):
    _fields_ = [("quad", ctypes.c_int32), ("Q", ctypes.c_int32), ("N", ctypes.c_int32),
                ("p0", ctypes.c_double)]


@dataclass
class Axis:
    """One axis of a mixed-quadrature velocity set (App. A)."""
    quad: int = HALF_HERMITE
    Q: int = 4
    N: int = -1          # < 0: min(20, Q - 1)
    p0: float = 1.0

    @property
    def V(self) -> int:
        return self.Q if self.quad == FULL_HERMITE else 2 * self.Q


def _axes(axes):
    arr = (_CAxis * len(axes))()
    for a, ax in enumerate(axes):
        arr[a] = _CAxis(ax.quad, ax.Q, ax.N if ax.N >= 0 else min(20, ax.Q - 1), ax.p0)
    return arr


_lib = None


def lib():
    """Load libhhlb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1708_03249_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        dp, vp = ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.hhlb_last_error.restype = ctypes.c_char_p
        L.hhlb_nodes.argtypes = [i32, i32, ctypes.c_double, dp, dp]
        L.hhlb_force_matrix.argtypes = [i32, i32, ctypes.c_double, dp]
        L.hhlb_equilibrium.argtypes = [i32, i32, i32] + [ctypes.c_double] * 4 + [dp]
        L.hhlb_create.argtypes = [ctypes.POINTER(_CChannel), i32, i32, vp, ctypes.POINTER(vp)]
        L.hhlb_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.hhlb_bind_workspace.argtypes = [vp, vp]
        L.hhlb_state_offsets.argtypes = [vp, ctypes.POINTER(i64)]
        L.hhlb_time_steps.argtypes = [vp, dp]
        L.hhlb_set_state.argtypes = [vp, vp, vp]
        L.hhlb_init_equilibrium.argtypes = [vp] + [ctypes.c_double] * 3
        L.hhlb_step.argtypes = [vp, i64]
        L.hhlb_get_state.argtypes = [vp, vp, vp]
        L.hhlb_moments.argtypes = [vp, vp, vp, vp]
        L.hhlb_diagnostics.argtypes = [vp, vp, vp, vp, vp]
        L.hhlb_launch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.hhlb_destroy.argtypes = [vp]
        L.hhlb_wide_equilibrium_count.argtypes = [vp, ctypes.POINTER(i64)]
        L.hhlb_equilibrium_ladder.argtypes = [vp, i32, ctypes.POINTER(i32), dp]
        L.hhlb_set_graph_steps.argtypes = [vp, i32]
        L.hhlb_set_tuning.argtypes = [vp, ctypes.POINTER(_CTuning)]
        L.hhlb_get_tuning.argtypes = [vp, ctypes.POINTER(_CTuning)]
        L.hhlb_autotune.argtypes = [vp, i32, ctypes.POINTER(_CTuning)]
        ap = ctypes.POINTER(_CAxis)
        L.hhlb_multi_nodes.argtypes = [ap, i32, dp, dp]
        L.hhlb_multi_workspace_bytes.argtypes = [ap, i32, i64, ctypes.POINTER(ctypes.c_size_t)]
        L.hhlb_multi_rhs.argtypes = [ap, i32, vp, i64, dp, ctypes.c_double, vp, vp, ctypes.c_size_t, vp]
        L.hhlb_multi_step.argtypes = [ap, i32, vp, i64, dp, ctypes.c_double, ctypes.c_double, i32, vp,
                                      ctypes.c_size_t, vp]
        L.hhlb_multi_step_noalloc.argtypes = [ap, i32, vp, i64, dp, ctypes.c_double, ctypes.c_double, i32, vp]
        for name in ("hhlb_multi_nodes", "hhlb_multi_workspace_bytes", "hhlb_multi_rhs", "hhlb_multi_step",
                     "hhlb_multi_step_noalloc"):
            getattr(L, name).restype = ctypes.c_int32
        for name in ("hhlb_nodes", "hhlb_force_matrix", "hhlb_equilibrium", "hhlb_create",
                     "hhlb_workspace_bytes", "hhlb_bind_workspace", "hhlb_state_offsets",
                     "hhlb_time_steps", "hhlb_set_state", "hhlb_init_equilibrium", "hhlb_step",
                     "hhlb_get_state", "hhlb_moments", "hhlb_diagnostics", "hhlb_launch_info",
                     "hhlb_destroy", "hhlb_set_graph_steps", "hhlb_set_tuning", "hhlb_get_tuning",
                     "hhlb_autotune", "hhlb_wide_equilibrium_count", "hhlb_equilibrium_ladder"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise HHLBError(st, lib().hhlb_last_error().decode())


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def nodes(quad: int, Q: int, p0: float = 1.0):
    V = Q if quad == FULL_HERMITE else 2 * Q
    p, w = np.zeros(V), np.zeros(V)
    _check(lib().hhlb_nodes(quad, Q, p0, _dptr(p), _dptr(w)))
    return p, w


def force_matrix(quad: int, Q: int, p0: float = 1.0):
    V = Q if quad == FULL_HERMITE else 2 * Q
    K = np.zeros((V, V))
    _check(lib().hhlb_force_matrix(quad, Q, p0, _dptr(K)))
    return K


def equilibrium(quad: int, Q: int, N: int, n: float, u: float, T: float, p0: float = 1.0):
    V = Q if quad == FULL_HERMITE else 2 * Q
    g = np.zeros(V)
    _check(lib().hhlb_equilibrium(quad, Q, N, p0, n, u, T, _dptr(g)))
    return g


def multi_nodes(axes):
    """App. A.1: momenta (d, V) and product weights (V,) of a mixed set."""
    V = int(np.prod([a.V for a in axes]))
    p, w = np.zeros((len(axes), V)), np.zeros(V)
    _check(lib().hhlb_multi_nodes(_axes(axes), len(axes), _dptr(p), _dptr(w)))
    return p, w


class MultiSolver:
    """The homogeneous mixed-quadrature system of App. A for npts points on
    one GPU: f is a (npts, V) float64 CUDA tensor the caller owns; the
    workspace (tables and two RK stage copies) comes from torch."""

    def __init__(self, axes, npts, F, Kn, stream=None):
        import torch
        self.axes, self.npts = list(axes), int(npts)
        self.F = np.ascontiguousarray(np.asarray(F, dtype=np.float64))
        assert self.F.shape == (len(self.axes),)
        self.Kn = float(Kn)
        self.V = int(np.prod([a.V for a in self.axes]))
        self._ax = _axes(self.axes)
        nb = ctypes.c_size_t()
        _check(lib().hhlb_multi_workspace_bytes(self._ax, len(self.axes), self.npts, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.stream = stream or torch.cuda.current_stream()

    def _f(self, f):
        import torch
        assert f.dtype == torch.float64 and f.is_cuda and f.is_contiguous() and f.numel() == self.npts * self.V
        return ctypes.c_void_p(f.data_ptr())

    def rhs(self, f, L):
        _check(lib().hhlb_multi_rhs(self._ax, len(self.axes), self._f(f), self.npts, _dptr(self.F), self.Kn,
                                    self._f(L), ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                    ctypes.c_void_p(self.stream.cuda_stream)))

    def step(self, f, dt, n_steps):
        _check(lib().hhlb_multi_step(self._ax, len(self.axes), self._f(f), self.npts, _dptr(self.F), self.Kn,
                                     float(dt), int(n_steps), ctypes.c_void_p(self.ws.data_ptr()),
                                     self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream)))


def multi_step_noalloc(axes, f, F, Kn, dt, n_steps, stream=None):
    """hhlb_multi_step_noalloc: n_steps RK-3 steps of the homogeneous
    mixed-quadrature system in place on f, a (npts, V) float64 CUDA tensor,
    with the library's static device scratch instead of a workspace."""
    import torch
    V = int(np.prod([a.V for a in axes]))
    assert f.dtype == torch.float64 and f.is_cuda and f.is_contiguous() and f.numel() % V == 0
    F = np.ascontiguousarray(np.asarray(F, dtype=np.float64))
    assert F.shape == (len(axes),)
    st = stream or torch.cuda.current_stream()
    _check(lib().hhlb_multi_step_noalloc(_axes(axes), len(axes), ctypes.c_void_p(f.data_ptr()),
                                         f.numel() // V, _dptr(F), float(Kn), float(dt), int(n_steps),
                                         ctypes.c_void_p(st.cuda_stream)))


class Solver:
    """Channels advanced on one GPU.  Device memory comes from torch."""

    def __init__(self, channels, device="cuda", stream=None, precision=FP64):
        import torch
        self.torch = torch
        self.channels = list(channels)
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.precision = int(precision)
        arr = (_CChannel * len(self.channels))(*[c._c() for c in self.channels])
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib().hhlb_create(arr, len(self.channels), self.precision,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        nb = ctypes.c_size_t()
        _check(lib().hhlb_workspace_bytes(self.h, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        _check(lib().hhlb_bind_workspace(self.h, ctypes.c_void_p(self._ws_ptr)))
        off = (ctypes.c_int64 * (len(self.channels) + 1))()
        _check(lib().hhlb_state_offsets(self.h, off))
        self.offsets = np.array(off[:], dtype=np.int64)
        dts = np.zeros(len(self.channels))
        _check(lib().hhlb_time_steps(self.h, _dptr(dts)))
        self.dt = dts
        self.has_chi = any(c.transverse_dof > 0 for c in self.channels)
        self.total = int(self.offsets[-1])
        self.cells = np.cumsum([0] + [c.Nx for c in self.channels])

    # -- state ------------------------------------------------------------
    def set_state(self, f, chi=None):
        f = f.contiguous()
        chi = chi.contiguous() if chi is not None else None
        assert f.dtype == self.torch.float64 and f.numel() == self.total
        _check(lib().hhlb_set_state(self.h, ctypes.c_void_p(f.data_ptr()),
                                    ctypes.c_void_p(chi.data_ptr() if chi is not None else 0)))

    def init_equilibrium(self, n0=1.0, u0=0.0, T0=1.0):
        _check(lib().hhlb_init_equilibrium(self.h, n0, u0, T0))

    def get_state(self):
        t = self.torch
        f = t.empty(self.total, dtype=t.float64, device=self.device)
        c = t.empty(self.total, dtype=t.float64, device=self.device)
        _check(lib().hhlb_get_state(self.h, ctypes.c_void_p(f.data_ptr()),
                                    ctypes.c_void_p(c.data_ptr())))
        return f, c

    def step(self, n_steps: int):
        _check(lib().hhlb_step(self.h, int(n_steps)))

    def set_tuning(self, graph_steps=0, class_streams=0, xcd_map=1, waves_per_window=2, step_fusion=0,
                   merge_classes=0):
        t = _CTuning(int(graph_steps), int(class_streams), int(xcd_map), int(waves_per_window),
                     int(step_fusion), int(merge_classes), 0.0)
        _check(lib().hhlb_set_tuning(self.h, ctypes.byref(t)))

    def tuning(self):
        t = _CTuning()
        _check(lib().hhlb_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, trial_steps: int = 10):
        """Time every launch configuration on these channels and keep the
        fastest (advances the state like warm-up steps); returns it."""
        t = _CTuning()
        _check(lib().hhlb_autotune(self.h, int(trial_steps), ctypes.byref(t)))
        return t.as_dict()

    def set_graph_steps(self, steps_per_graph: int):
        """Steps per replayed HIP graph; 0 = direct launches."""
        _check(lib().hhlb_set_graph_steps(self.h, int(steps_per_graph)))

    def moments(self):
        t = self.torch
        nc = int(self.cells[-1])
        n, u, T = (t.empty(nc, dtype=t.float64, device=self.device) for _ in range(3))
        _check(lib().hhlb_moments(self.h, ctypes.c_void_p(n.data_ptr()),
                                  ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(T.data_ptr())))
        return n, u, T

    def diagnostics(self, residual: bool = False):
        """(n_wall [n_ch, 2], mass [n_ch], nonfinite [1]) as device tensors,
        plus the residual [n_ch] when residual=True (one extra stage launch)."""
        t = self.torch
        nch = len(self.channels)
        nw = t.empty(2 * nch, dtype=t.float64, device=self.device)
        mass = t.empty(nch, dtype=t.float64, device=self.device)
        res = t.empty(nch, dtype=t.float64, device=self.device) if residual else None
        bad = t.empty(1, dtype=t.int32, device=self.device)
        _check(lib().hhlb_diagnostics(self.h, ctypes.c_void_p(nw.data_ptr()),
                                      ctypes.c_void_p(mass.data_ptr()),
                                      ctypes.c_void_p(res.data_ptr() if residual else 0),
                                      ctypes.c_void_p(bad.data_ptr())))
        if residual:
            return nw.view(nch, 2), mass, bad, res
        return nw.view(nch, 2), mass, bad

    def wide_equilibrium_count(self) -> int:
        """Equilibrium evaluations whose |u|/sqrt(T) lay beyond the correction
        ladder's calibrated range (and ran the composite rule); syncs."""
        c = ctypes.c_int64()
        _check(lib().hhlb_wide_equilibrium_count(self.h, ctypes.byref(c)))
        return c.value

    def equilibrium_ladder(self, channel: int = 0):
        """(counts[8], reach[8]) of the channel's correction ladder."""
        n = (ctypes.c_int32 * 8)()
        r = np.zeros(8)
        _check(lib().hhlb_equilibrium_ladder(self.h, int(channel), n, _dptr(r)))
        return list(n), r

    def launch_info(self):
        a, b = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().hhlb_launch_info(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # -- helpers ----------------------------------------------------------
    def channel_view(self, flat, c: int):
        """(V, Nx) view of channel c inside a flat state array."""
        ch = self.channels[c]
        return flat[self.offsets[c]:self.offsets[c + 1]].view(ch.V, ch.Nx)

    def close(self):
        if getattr(self, "h", None):
            lib().hhlb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
