"""MI355X-native seismic saliency (Shafiq, Long, Di, AlRegib, ACI 2021, Sec. 2).

Thin PyTorch-facing binding of libsal: it checks tensors, passes their device
pointers and torch's current HIP stream to the C ABI, and nothing else -- all
arithmetic runs in the library's HIP kernels.  There is no CPU path: calling
any operation without the built library or without a GPU raises.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _lib

__all__ = ["Config", "init", "local_spectra", "project", "center_surround", "fuse", "saliency", "backward",
           "SaliencyFn", "grid_shape", "fuse_groups", "fuse_workspace_size", "backward_workspace_size", "adapt_weights",
           "line_template", "Plan"]


def _torch():
    import torch
    return torch


def grid_shape(shape, s):
    return tuple(-(-int(N) // int(s)) for N in shape)


_ready = set()


def init():
    """Upload libsal's constant tables to the current device (sal_init); needed once per
    device before any call is captured in a graph.  The operations below call it by
    themselves outside a capture."""
    torch = _torch()
    dev = torch.cuda.current_device()
    if dev not in _ready:
        _lib.check(_lib.load().sal_init())
        _ready.add(dev)


def _stream():
    torch = _torch()
    if torch.cuda.current_device() not in _ready:
        if torch.cuda.is_current_stream_capturing():
            raise RuntimeError("call paper_2201_06174_amd.init() on this device before capturing a graph")
        init()
    return ctypes_void(torch.cuda.current_stream().cuda_stream)


def ctypes_void(v):
    import ctypes
    return ctypes.c_void_p(int(v))


def _ptr(t):
    return None if t is None else ctypes_void(t.data_ptr())


def _need(t, dtype, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


@dataclass
class Config:
    """Parameters of the method besides the volume (Sec. 2)."""
    n: int = 8
    s: int = 1
    window: str = "hann"
    precision: str = "fp32"
    # "magnitude" (mean |F_m|) or "energy" (mean |F_m|^2; fp32 only)
    feature: str = "magnitude"
    offsets: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int32))
    weights: Optional[np.ndarray] = None
    literal: bool = False
    fusion: str = "equal"
    wfix: Optional[tuple] = None
    delta: float = 0.0
    # per-plane stencils [(offsets, weights or None)] for t, x, y (replace offsets/weights)
    planes: Optional[list] = None
    # re-adapt the fusion weights every `sections` grid inline sections (0: one fit)
    sections: int = 0
    # sequential rules (fusion "lms", "nlms", "rls"; wfix = starting weights, delta = RLS P0^-1)
    mu: float = 0.5
    eps: float = 1e-6
    lam: float = 1.0
    passes: int = 1


def line_template(direction, length, sigma):
    """Graded directional line template (offsets [2L][3], weights [2L]) for Config.offsets or
    one entry of Config.planes."""
    return _lib.line_template(direction, length, sigma)


def fuse_groups(ILg, sections=0):
    """Number of weight groups of the fusion over ILg grid inline planes."""
    return int(_lib.load().sal_fuse_groups(_lib.make_fusion("equal", None, 0.0, sections), int(ILg)))


def local_spectra(V, centers, n, window="hann"):
    """F[cnt][n][n][n] complex64 at voxel centres (device int32 [cnt][3])."""
    torch = _torch()
    _need(V, torch.float32, "V")
    _need(centers, torch.int32, "centers")
    if V.dim() != 3:
        raise ValueError("V must be [T][IL][XL]")
    if centers.dim() != 2 or centers.shape[1] != 3:
        raise ValueError("centers must be [cnt][3], got %s" % (tuple(centers.shape),))
    cnt = centers.shape[0]
    F = torch.empty((cnt, n, n, n, 2), dtype=torch.float32, device=V.device)
    spec = _lib.make_spec(n, 1, window)
    T, IL, XL = V.shape
    _lib.check(_lib.load().sal_local_spectra(_ptr(V), T, IL, XL, spec, _ptr(centers), cnt, _ptr(F), _stream()))
    return torch.view_as_complex(F)


def project(V, n, s, window="hann", precision="fp32", feature="magnitude"):
    """Features E[3][Tg][ILg][XLg] (planes t, x = XL, y = IL)."""
    torch = _torch()
    _need(V, torch.float32, "V")
    if V.dim() != 3:
        raise ValueError("V must be [T][IL][XL]")
    T, IL, XL = V.shape
    E = torch.empty((3,) + grid_shape(V.shape, s), dtype=torch.float32, device=V.device)
    spec = _lib.make_spec(n, s, window, precision, feature)
    _lib.check(_lib.load().sal_project(_ptr(V), T, IL, XL, spec, _ptr(E), _stream()))
    return E


def center_surround(E, s, offsets, weights=None, literal=False, planes=None):
    torch = _torch()
    _need(E, torch.float32, "E")
    if E.dim() != 4 or E.shape[0] != 3:
        raise ValueError("E must be [3][Tg][ILg][XLg]")
    Sm = torch.empty_like(E)
    st, keep = _lib.make_stencil(offsets, weights, literal, planes)
    _lib.check(_lib.load().sal_center_surround(_ptr(E), E.shape[1], E.shape[2], E.shape[3], s, st, _ptr(Sm),
                                               _stream()))
    del keep
    return Sm


def fuse_workspace_size(grid, sections=0, mode="equal"):
    f = _lib.make_fusion(mode, None, 0.0, sections)
    return int(_lib.load().sal_fuse_workspace_size(grid[0], grid[1], grid[2], f))


def _fusion(cfg):
    return _lib.make_fusion(cfg.fusion, cfg.wfix, cfg.delta, cfg.sections, cfg.mu, cfg.eps, cfg.lam, cfg.passes)


def fuse(Sm, shape, s, mode="equal", wfix=None, delta=0.0, D=None, mask=None, ws=None, sections=0, mu=0.5,
         eps=1e-6, lam=1.0, passes=1):
    """(S[T][IL][XL], W float64: W_t, W_x, W_y, fallback flag -- shape [4] without sections,
    [K][4] with re-adaptation every `sections` inline sections).  Modes equal, fixed,
    adapt_ls, and the sequential lms, nlms, rls (wfix: their starting weights)."""
    torch = _torch()
    _need(Sm, torch.float32, "Sm")
    if Sm.dim() != 4 or Sm.shape[0] != 3:
        raise ValueError("Sm must be [3][Tg][ILg][XLg], got %s" % (tuple(Sm.shape),))
    grid = tuple(Sm.shape[1:])
    if grid != grid_shape(shape, s):
        raise ValueError("Sm grid %s does not match ceil(%s / %d)" % (grid, tuple(shape), s))
    if D is not None:
        _need(D, torch.float32, "D", grid)
    if mask is not None:
        _need(mask, torch.uint8, "mask", grid)
    T, IL, XL = shape
    S = torch.empty((T, IL, XL), dtype=torch.float32, device=Sm.device)
    f = _lib.make_fusion(mode, wfix, delta, sections, mu, eps, lam, passes)
    K = int(_lib.load().sal_fuse_groups(f, grid[1]))
    W = torch.empty((K, 4) if sections else (4,), dtype=torch.float64, device=Sm.device)
    nbytes = fuse_workspace_size(grid, sections, mode)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=Sm.device)
    _lib.check(_lib.load().sal_fuse(_ptr(Sm), grid[0], grid[1], grid[2], f, _ptr(D), _ptr(mask), T, IL, XL, s,
                                    _ptr(W), _ptr(S), _ptr(ws), ws.numel(), _stream()))
    return S, W


def saliency(V, cfg: Config, D=None, mask=None):
    """Whole forward path: returns dict(E, Sm, S, W)."""
    E = project(V, cfg.n, cfg.s, cfg.window, cfg.precision, cfg.feature)
    Sm = center_surround(E, cfg.s, cfg.offsets, cfg.weights, cfg.literal, cfg.planes)
    S, W = fuse(Sm, tuple(V.shape), cfg.s, cfg.fusion, cfg.wfix, cfg.delta, D, mask, sections=cfg.sections,
                mu=cfg.mu, eps=cfg.eps, lam=cfg.lam, passes=cfg.passes)
    return {"E": E, "Sm": Sm, "S": S, "W": W}


def adapt_weights(Sm, cfg: Config, D, mask=None, cap=0):
    """The sequential LMS / NLMS / RLS weights (cfg.fusion "lms", "nlms" or "rls") and their
    learning curve: (W [K][4] float64, err2 [K][cap] float32 squared a priori errors in update
    order, count [K] int64 samples per pass)."""
    torch = _torch()
    _need(Sm, torch.float32, "Sm")
    if Sm.dim() != 4 or Sm.shape[0] != 3:
        raise ValueError("Sm must be [3][Tg][ILg][XLg], got %s" % (tuple(Sm.shape),))
    grid = tuple(Sm.shape[1:])
    _need(D, torch.float32, "D", grid)
    if mask is not None:
        _need(mask, torch.uint8, "mask", grid)
    f = _fusion(cfg)
    K = int(_lib.load().sal_fuse_groups(f, grid[1]))
    W = torch.empty((K, 4), dtype=torch.float64, device=Sm.device)
    err = torch.empty((K, max(int(cap), 1)), dtype=torch.float32, device=Sm.device)
    cnt = torch.empty(K, dtype=torch.int64, device=Sm.device)
    nbytes = int(_lib.load().sal_fuse_workspace_size(grid[0], grid[1], grid[2], f))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=Sm.device)
    _lib.check(_lib.load().sal_adapt_weights(_ptr(Sm), grid[0], grid[1], grid[2], f, _ptr(D), _ptr(mask), _ptr(W),
                                             _ptr(err) if cap else None, int(cap), _ptr(cnt), _ptr(ws), ws.numel(),
                                             _stream()))
    return W, err[:, :cap], cnt


def backward_workspace_size(shape, n, s, window="hann", precision="fp32", sections=0):
    spec = _lib.make_spec(n, s, window, precision)
    f = _lib.make_fusion("equal", None, 0.0, sections)
    return int(_lib.load().sal_backward_workspace_size(shape[0], shape[1], shape[2], spec, f))


def backward(V, cfg: Config, E, Sm, W, gS, D=None, mask=None):
    """gV = d(sum gS * S)/dV through the hand-written adjoint (spectra recomputed)."""
    torch = _torch()
    _need(V, torch.float32, "V")
    if V.dim() != 3:
        raise ValueError("V must be [T][IL][XL]")
    grid = grid_shape(V.shape, cfg.s)
    _need(gS, torch.float32, "gS", tuple(V.shape))
    _need(E, torch.float32, "E", (3,) + grid)
    _need(Sm, torch.float32, "Sm", (3,) + grid)
    K = fuse_groups(grid[1], cfg.sections)
    _need(W, torch.float64, "W", (K, 4) if cfg.sections else (4,))
    if D is not None:
        _need(D, torch.float32, "D", grid)
    if mask is not None:
        _need(mask, torch.uint8, "mask", grid)
    T, IL, XL = V.shape
    gV = torch.empty_like(V)
    spec = _lib.make_spec(cfg.n, cfg.s, cfg.window, cfg.precision, cfg.feature)
    st, keep = _lib.make_stencil(cfg.offsets, cfg.weights, cfg.literal, cfg.planes)
    f = _fusion(cfg)
    nbytes = backward_workspace_size(V.shape, cfg.n, cfg.s, cfg.window, cfg.precision, cfg.sections)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=V.device)
    _lib.check(_lib.load().sal_backward(_ptr(V), T, IL, XL, spec, st, f, _ptr(E), _ptr(Sm), _ptr(W), _ptr(D),
                                        _ptr(mask), _ptr(gS), _ptr(gV), _ptr(ws), ws.numel(), _stream()))
    del keep
    return gV


def _make_fn():
    torch = _torch()

    class SaliencyFn(torch.autograd.Function):
        """S = saliency(V); backward through libsal's adjoint.  Saves V, E, S_m and W
        (never the local spectra, which the adjoint recomputes)."""

        @staticmethod
        def forward(ctx, V, cfg, D=None, mask=None):
            r = saliency(V, cfg, D, mask)
            ctx.cfg = cfg
            ctx.save_for_backward(V, r["E"], r["Sm"], r["W"], D, mask)
            return r["S"]

        @staticmethod
        def backward(ctx, gS):
            V, E, Sm, W, D, mask = ctx.saved_tensors
            gV = backward(V, ctx.cfg, E, Sm, W, gS.contiguous(), D, mask)
            return gV, None, None, None

    return SaliencyFn


class _Lazy:
    _fn = None

    def __getattr__(self, item):
        if _Lazy._fn is None:
            _Lazy._fn = _make_fn()
        return getattr(_Lazy._fn, item)


SaliencyFn = _Lazy()


class Plan:
    """The whole forward path over many volumes as one captured graph of
    persistent kernels (libsal's sal_plan_*).  Members: dicts with keys V
    (device float32 [T][IL][XL]), cfg (Config), and optionally D, mask.  The
    plan allocates each member's outputs; launch() runs the batch on the
    current stream, output(i) returns member i's E, Sm, S and W."""

    def __init__(self, members, autotune=False, graph=True):
        import ctypes
        torch = _torch()
        self._keep = []
        self._out = []
        arr = (_lib.SalBatchItem * len(members))()
        for i, m in enumerate(members):
            V, cfg = m["V"], m["cfg"]
            _need(V, torch.float32, "V")
            D, mask = m.get("D"), m.get("mask")
            grid = grid_shape(V.shape, cfg.s)
            out = {"E": torch.empty((3,) + grid, dtype=torch.float32, device=V.device),
                   "Sm": torch.empty((3,) + grid, dtype=torch.float32, device=V.device),
                   "S": torch.empty(tuple(V.shape), dtype=torch.float32, device=V.device),
                   "W": torch.empty(4, dtype=torch.float64, device=V.device)}
            self._out.append(out)
            st, keep = _lib.make_stencil(cfg.offsets, cfg.weights, cfg.literal, cfg.planes)
            self._keep.append((V, D, mask, keep))
            it = arr[i]
            it.V = V.data_ptr()
            it.T, it.IL, it.XL = V.shape
            it.spec = _lib.make_spec(cfg.n, cfg.s, cfg.window, cfg.precision, cfg.feature)
            it.stencil = st
            it.fusion = _fusion(cfg)
            it.D = None if D is None else _need(D, torch.float32, "D", grid).data_ptr()
            it.mask = None if mask is None else _need(mask, torch.uint8, "mask", grid).data_ptr()
            it.E_out = out["E"].data_ptr()
            it.Sm_out = out["Sm"].data_ptr()
            it.W_out = out["W"].data_ptr()
            it.S_out = out["S"].data_ptr()
        init()
        flags = (_lib.PLAN_AUTOTUNE if autotune else 0) | (0 if graph else _lib.PLAN_NO_GRAPH)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().sal_plan_create(arr, len(members), flags, ctypes.byref(h)))
        self._h = h

    def launch(self):
        _lib.check(_lib.load().sal_plan_launch(self._h, _stream()))

    def output(self, i):
        return self._out[i]

    def status(self):
        """(number of members whose adapted fit fell back to equal weights, lowest such member
        or -1), after the launches enqueued so far (waits for the current stream)."""
        import ctypes
        c, f = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(_lib.load().sal_plan_status(self._h, _stream(), ctypes.byref(c), ctypes.byref(f)))
        return int(c.value), int(f.value)

    def describe(self):
        return _lib.load().sal_plan_describe(self._h).decode()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().sal_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
