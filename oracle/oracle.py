"""FP64 CPU oracle of the seismic saliency hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product library never does.

This is a thin ctypes binding over ``sal_oracle.c`` (plain C, FP64, OpenMP):
argument marshalling only, all arithmetic lives in the C file.  It follows
Shafiq, Long, Di, AlRegib (ACI 2021), Section 2:

* local 3D DFT of each window (Sec. 2 step 1, Eq. 2) -- ``local_spectra``;
* spectral projection and features E_m (Eq. 1, third step), as the mean of
  |F_m| or of the energy |F_m|^2 -- ``features``;
* directional center-surround S_m (Eq. 3) -- ``dcs``, ``saliency_at``;
* fusion weights and the combined map S (Eq. 4) -- ``fusion_weights``,
  ``combine``; the sequential LMS / NLMS / RLS weights and their learning
  curve -- ``adapt_sequential``; with re-adaptation every N inline sections
  ``fusion_weights_sections``, ``combine_sections``;
* per-plane stencils and graded line templates (Sec. 2 step 4, Fig. 4) --
  ``dcs_planes``, ``line_template``;
* the adjoint of the whole chain -- ``backward``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sal_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

WINDOWS = {"hann": 0, "rect": 1}
FEATURES = {"magnitude": 0, "energy": 1}
FUSION_MODES = {"equal": 0, "fixed": 1, "adapt_ls": 2}


def build(force: bool = True) -> str:
    """Compile liboracle.so next to the source (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _i64(v):
    return ctypes.c_int64(int(v))


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _nthreads(nthreads):
    return ctypes.c_int(0 if nthreads is None else int(nthreads))


def _vol(V):
    V = np.ascontiguousarray(V, dtype=np.float32)
    if V.ndim != 3:
        raise ValueError("V must be [T][IL][XL]")
    return V


def window(n: int, kind="hann") -> np.ndarray:
    h = np.zeros(n, np.float64)
    _check(_load().orc_window(ctypes.c_int(n), ctypes.c_int(WINDOWS.get(kind, kind)), _p(h)), "window")
    return h


def local_spectra(V, n: int, kind, centers) -> np.ndarray:
    """Unshifted spectra F[cnt][n][n][n] (complex128) at voxel centres [cnt][3]."""
    V = _vol(V)
    c = np.ascontiguousarray(centers, dtype=np.int64).reshape(-1, 3)
    F = np.zeros((c.shape[0], n, n, n, 2), np.float64)
    rc = _load().orc_local_spectra(_p(V), _i64(V.shape[0]), _i64(V.shape[1]), _i64(V.shape[2]), ctypes.c_int(n),
                                   ctypes.c_int(WINDOWS.get(kind, kind)), _p(c), _i64(c.shape[0]), _p(F))
    _check(rc, "local_spectra")
    return F[..., 0] + 1j * F[..., 1]


def grid_shape(shape, s):
    return tuple(-(-int(N) // int(s)) for N in shape)


def features(V, n: int, s: int, kind="hann", nthreads=None, feature="magnitude") -> np.ndarray:
    """E[3][Tg][ILg][XLg] in FP64 (planes t, x=XL, y=IL); feature "magnitude" (mean |F_m|) or
    "energy" (mean |F_m|^2)."""
    V = _vol(V)
    gs = grid_shape(V.shape, s)
    E = np.zeros((3,) + gs, np.float64)
    rc = _load().orc_features_ex(_p(V), _i64(V.shape[0]), _i64(V.shape[1]), _i64(V.shape[2]), ctypes.c_int(n),
                                 ctypes.c_int(s), ctypes.c_int(WINDOWS.get(kind, kind)),
                                 ctypes.c_int(FEATURES[feature]), _p(E), _nthreads(nthreads))
    _check(rc, "features")
    return E


def features_at(V, n: int, s: int, kind, g, nthreads=None, feature="magnitude") -> np.ndarray:
    """E at grid points g[cnt][3]; returns [cnt][3]."""
    V = _vol(V)
    g = np.ascontiguousarray(g, dtype=np.int64).reshape(-1, 3)
    E = np.zeros((g.shape[0], 3), np.float64)
    rc = _load().orc_features_at_ex(_p(V), _i64(V.shape[0]), _i64(V.shape[1]), _i64(V.shape[2]), ctypes.c_int(n),
                                    ctypes.c_int(s), ctypes.c_int(WINDOWS.get(kind, kind)),
                                    ctypes.c_int(FEATURES[feature]), _p(g), _i64(g.shape[0]), _p(E),
                                    _nthreads(nthreads))
    _check(rc, "features_at")
    return E


def default_weights(offsets) -> np.ndarray:
    off = np.ascontiguousarray(offsets, dtype=np.int32).reshape(-1, 3)
    w = np.zeros(off.shape[0], np.float64)
    _check(_load().orc_default_weights(ctypes.c_int(off.shape[0]), _p(off), _p(w)), "default_weights")
    return w


def _stencil(offsets, weights):
    off = np.ascontiguousarray(offsets, dtype=np.int32).reshape(-1, 3)
    w = default_weights(off) if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if w.shape != (off.shape[0],):
        raise ValueError("one weight per offset")
    return off, w


def dcs(E, s: int, offsets, weights=None, literal=False) -> np.ndarray:
    """S_m on the grid from E (both [3][Tg][ILg][XLg])."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    off, w = _stencil(offsets, weights)
    S = np.zeros_like(E)
    rc = _load().orc_dcs(_p(E), _i64(E.shape[1]), _i64(E.shape[2]), _i64(E.shape[3]), ctypes.c_int(s),
                         ctypes.c_int(off.shape[0]), _p(off), _p(w), ctypes.c_int(int(bool(literal))), _p(S))
    _check(rc, "dcs")
    return S


def line_template(direction, length: int, sigma: float):
    """(offsets[2L][3], weights[2L]): graded line template along `direction`."""
    d = np.ascontiguousarray(direction, dtype=np.int32).reshape(3)
    off = np.zeros((2 * length, 3), np.int32)
    w = np.zeros(2 * length, np.float64)
    _check(_load().orc_line_template(_p(d), ctypes.c_int(int(length)), ctypes.c_double(sigma), _p(off), _p(w)),
           "line_template")
    return off, w


def _planes(planes):
    """Per-plane stencils [(offsets, weights|None)] * 3 -> (q3, offsets, weights) concatenated."""
    if len(planes) != 3:
        raise ValueError("one stencil per plane (t, x, y)")
    offs, ws = [], []
    for off, w in planes:
        o, ww = _stencil(off, w)
        offs.append(o)
        ws.append(ww)
    q3 = np.array([o.shape[0] for o in offs], np.int32)
    return q3, np.ascontiguousarray(np.concatenate(offs), np.int32), np.ascontiguousarray(np.concatenate(ws))


def dcs_planes(E, s: int, planes, literal=False) -> np.ndarray:
    """S_m with a stencil per plane: planes = [(offsets, weights or None)] for t, x, y."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    q3, off, w = _planes(planes)
    S = np.zeros_like(E)
    rc = _load().orc_dcs_planes(_p(E), _i64(E.shape[1]), _i64(E.shape[2]), _i64(E.shape[3]), ctypes.c_int(s),
                                _p(q3), _p(off), _p(w), ctypes.c_int(int(bool(literal))), _p(S))
    _check(rc, "dcs_planes")
    return S


def fuse_groups(ILg: int, sections: int) -> int:
    f = _load().orc_fuse_groups
    f.restype = ctypes.c_int64
    return int(f(_i64(ILg), _i64(sections)))


def fusion_weights_sections(Sm, sections: int, D=None, mask=None, mode="equal", wfix=None, delta=0.0):
    """(W[K][3], fallback[K], stats[K][11]) with re-adaptation every `sections` inline sections."""
    Sm = np.ascontiguousarray(Sm, dtype=np.float64)
    _, Tg, ILg, XLg = Sm.shape
    K = fuse_groups(ILg, sections)
    Dp = None if D is None else np.ascontiguousarray(D, dtype=np.float32).reshape(-1)
    Mp = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    wf = None if wfix is None else np.ascontiguousarray(wfix, dtype=np.float64)
    W = np.zeros((K, 3), np.float64)
    fb = np.zeros(K, np.int32)
    st = np.zeros((K, 11), np.float64)
    rc = _load().orc_fusion_weights_sections(_p(Sm), _i64(Tg), _i64(ILg), _i64(XLg), _p(Dp), _p(Mp),
                                             ctypes.c_int(FUSION_MODES.get(mode, mode)), _p(wf),
                                             ctypes.c_double(delta), _i64(sections), _p(W), _p(fb), _p(st))
    _check(rc, "fusion_weights_sections")
    return W, fb, st


ADAPT_RULES = {"lms": 0, "nlms": 1, "rls": 2}


def adapt_sequential(Sm, D, mask=None, rule="nlms", mu=0.5, eps=1e-6, lam=1.0, delta=1.0, w0=(1 / 3, 1 / 3, 1 / 3),
                     passes=1, sections=0, cap=0):
    """(W[K][3], count[K], err2[K][cap]): the sequential LMS / NLMS / RLS weights over the masked
    grid points in memory order, and the squared a priori errors in update order."""
    Sm = np.ascontiguousarray(Sm, dtype=np.float64)
    _, Tg, ILg, XLg = Sm.shape
    K = fuse_groups(ILg, sections)
    Dp = np.ascontiguousarray(D, dtype=np.float32).reshape(-1)
    Mp = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    w = np.ascontiguousarray(w0, dtype=np.float64)
    W = np.zeros((K, 3), np.float64)
    cnt = np.zeros(K, np.int64)
    err = np.zeros((K, max(cap, 1)), np.float64)
    rc = _load().orc_adapt_sequential(_p(Sm), _i64(Tg), _i64(ILg), _i64(XLg), _p(Dp), _p(Mp),
                                      ctypes.c_int(ADAPT_RULES[rule]), ctypes.c_double(mu), ctypes.c_double(eps),
                                      ctypes.c_double(lam), ctypes.c_double(delta), _p(w), ctypes.c_int(passes),
                                      _i64(sections), _p(W), _p(cnt), _p(err) if cap else None, _i64(cap))
    _check(rc, "adapt_sequential")
    return W, cnt, err[:, :cap]


def combine_sections(Sm, W, sections: int, shape, s: int) -> np.ndarray:
    Sm = np.ascontiguousarray(Sm, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(-1, 3)
    T, IL, XL = shape
    S = np.zeros((T, IL, XL), np.float64)
    rc = _load().orc_combine_sections(_p(Sm), _i64(Sm.shape[1]), _i64(Sm.shape[2]), _i64(Sm.shape[3]), _p(W),
                                      _i64(sections), _i64(T), _i64(IL), _i64(XL), ctypes.c_int(s), _p(S))
    _check(rc, "combine_sections")
    return S


def saliency_at(V, n, s, kind, offsets, weights, literal, g, nthreads=None):
    """(S_m[cnt][3], E[cnt][3]) at grid points g, features recomputed from V."""
    V = _vol(V)
    off, w = _stencil(offsets, weights)
    g = np.ascontiguousarray(g, dtype=np.int64).reshape(-1, 3)
    Sm = np.zeros((g.shape[0], 3), np.float64)
    E = np.zeros((g.shape[0], 3), np.float64)
    rc = _load().orc_saliency_at(_p(V), _i64(V.shape[0]), _i64(V.shape[1]), _i64(V.shape[2]), ctypes.c_int(n),
                                 ctypes.c_int(s), ctypes.c_int(WINDOWS.get(kind, kind)), ctypes.c_int(off.shape[0]),
                                 _p(off), _p(w), ctypes.c_int(int(bool(literal))), _p(g), _i64(g.shape[0]), _p(Sm),
                                 _p(E), _nthreads(nthreads))
    _check(rc, "saliency_at")
    return Sm, E


def saliency_inline_plane(V, n, s, kind, offsets, weights, literal, il_g, nthreads=None):
    """(E, S_m) on one grid inline plane il_g, both [3][Tg][XLg], for volumes too large for
    the full-grid oracle: E on the grid planes within the stencil's inline reach (features_at)
    and the center-surround of that sub-grid (dcs).  A neighbour of plane il_g lies inside
    the sub-grid exactly when it lies inside the full grid, so S_m on il_g is exact."""
    V = _vol(V)
    off, w = _stencil(offsets, weights)
    Tg, ILg, XLg = grid_shape(V.shape, s)
    r = int(np.max(np.abs(off[:, 1]))) // s
    lo, hi = max(0, il_g - r), min(ILg, il_g + r + 1)
    t, i, x = np.meshgrid(np.arange(Tg), np.arange(lo, hi), np.arange(XLg), indexing="ij")
    g = np.stack([t.ravel(), i.ravel(), x.ravel()], 1).astype(np.int64)
    E = features_at(V, n, s, kind, g, nthreads).T.reshape(3, Tg, hi - lo, XLg)
    Sm = dcs(E, s, off, w, literal)
    return np.ascontiguousarray(E[:, :, il_g - lo, :]), np.ascontiguousarray(Sm[:, :, il_g - lo, :])


def fusion_weights(Sm, D=None, mask=None, mode="equal", wfix=None, delta=0.0):
    """(W[3], fallback, stats[11]) -- Eq. 4 weights; stats only for adapt_ls."""
    Sm = np.ascontiguousarray(Sm, dtype=np.float64)
    G = Sm[0].size
    Dp = None if D is None else np.ascontiguousarray(D, dtype=np.float32).reshape(-1)
    Mp = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    wf = None if wfix is None else np.ascontiguousarray(wfix, dtype=np.float64)
    W = np.zeros(3, np.float64)
    st = np.zeros(11, np.float64)
    fb = ctypes.c_int(0)
    rc = _load().orc_fusion_weights(_p(Sm), _i64(G), _p(Dp), _p(Mp), ctypes.c_int(FUSION_MODES.get(mode, mode)),
                                    _p(wf), ctypes.c_double(delta), _p(W), ctypes.byref(fb), _p(st))
    _check(rc, "fusion_weights")
    return W, int(fb.value), st


def combine(Sm, W, shape, s: int) -> np.ndarray:
    Sm = np.ascontiguousarray(Sm, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    T, IL, XL = shape
    S = np.zeros((T, IL, XL), np.float64)
    rc = _load().orc_combine(_p(Sm), _i64(Sm.shape[1]), _i64(Sm.shape[2]), _i64(Sm.shape[3]), _p(W), _i64(T),
                             _i64(IL), _i64(XL), ctypes.c_int(s), _p(S))
    _check(rc, "combine")
    return S


@dataclass
class Params:
    """Everything the method takes besides V (Sec. 2)."""
    n: int = 8
    s: int = 1
    window: str = "hann"
    offsets: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int32))
    weights: Optional[np.ndarray] = None
    literal: bool = False
    fusion: str = "equal"
    wfix: Optional[np.ndarray] = None
    delta: float = 0.0
    D: Optional[np.ndarray] = None
    mask: Optional[np.ndarray] = None
    # per-plane stencils [(offsets, weights or None)] for t, x, y (replace offsets/weights)
    planes: Optional[list] = None
    # re-adaptation every `sections` grid inline sections (0: one fit)
    sections: int = 0
    # "magnitude" (mean |F_m|, Sec. 2 third step) or "energy" (mean |F_m|^2)
    feature: str = "magnitude"


def _plane_stencils(p: Params):
    if p.planes is not None:
        return _planes(p.planes)
    off, w = _stencil(p.offsets, p.weights)
    return (np.array([off.shape[0]] * 3, np.int32), np.ascontiguousarray(np.concatenate([off] * 3), np.int32),
            np.ascontiguousarray(np.concatenate([w] * 3)))


def forward(V, p: Params, nthreads=None) -> dict:
    """E, S_m, W, fallback flag and S for the whole volume (W [3] and an int flag without
    sections, W [K][3] and flags [K] with them)."""
    V = _vol(V)
    E = features(V, p.n, p.s, p.window, nthreads, p.feature)
    if p.planes is not None:
        Sm = dcs_planes(E, p.s, p.planes, p.literal)
    else:
        Sm = dcs(E, p.s, p.offsets, p.weights, p.literal)
    if p.sections:
        W, fb, st = fusion_weights_sections(Sm, p.sections, p.D, p.mask, p.fusion, p.wfix, p.delta)
        S = combine_sections(Sm, W, p.sections, V.shape, p.s)
    else:
        W, fb, st = fusion_weights(Sm, p.D, p.mask, p.fusion, p.wfix, p.delta)
        S = combine(Sm, W, V.shape, p.s)
    return {"E": E, "Sm": Sm, "W": W, "fallback": fb, "stats": st, "S": S}


def backward(V, p: Params, gS, nthreads=None):
    """(gV, W, fallback): gradient of sum(gS * S) with respect to V (W and fallback shaped as
    in forward)."""
    V = _vol(V)
    q3, off, w = _plane_stencils(p)
    gS = np.ascontiguousarray(gS, dtype=np.float32)
    if gS.shape != V.shape:
        raise ValueError("gS must match V")
    Dp = None if p.D is None else np.ascontiguousarray(p.D, dtype=np.float32).reshape(-1)
    Mp = None if p.mask is None else np.ascontiguousarray(p.mask, dtype=np.uint8).reshape(-1)
    wf = None if p.wfix is None else np.ascontiguousarray(p.wfix, dtype=np.float64)
    K = fuse_groups(grid_shape(V.shape, p.s)[1], p.sections)
    gV = np.zeros(V.shape, np.float64)
    W = np.zeros((K, 3), np.float64)
    fb = np.zeros(K, np.int32)
    rc = _load().orc_backward_ex(_p(V), _i64(V.shape[0]), _i64(V.shape[1]), _i64(V.shape[2]), ctypes.c_int(p.n),
                                 ctypes.c_int(p.s), ctypes.c_int(WINDOWS.get(p.window, p.window)),
                                 ctypes.c_int(FEATURES[p.feature]), _p(q3), _p(off),
                                 _p(w), ctypes.c_int(int(bool(p.literal))),
                                 ctypes.c_int(FUSION_MODES.get(p.fusion, p.fusion)), _p(wf), ctypes.c_double(p.delta),
                                 _p(Dp), _p(Mp), _i64(p.sections), _p(gS), _p(gV), _p(W), _p(fb),
                                 _nthreads(nthreads))
    _check(rc, "backward")
    if p.sections:
        return gV, W, fb
    return gV, W[0], int(fb[0])


def backward_at(V, p: Params, gS, pts, nthreads=None) -> np.ndarray:
    """gV at voxels pts[cnt][3] for equal or fixed fusion."""
    V = _vol(V)
    off, w = _stencil(p.offsets, p.weights)
    gS = np.ascontiguousarray(gS, dtype=np.float32)
    pts = np.ascontiguousarray(pts, dtype=np.int64).reshape(-1, 3)
    wf = None if p.wfix is None else np.ascontiguousarray(p.wfix, dtype=np.float64)
    gV = np.zeros(pts.shape[0], np.float64)
    rc = _load().orc_backward_at(_p(V), _i64(V.shape[0]), _i64(V.shape[1]), _i64(V.shape[2]), ctypes.c_int(p.n),
                                 ctypes.c_int(p.s), ctypes.c_int(WINDOWS.get(p.window, p.window)),
                                 ctypes.c_int(off.shape[0]), _p(off), _p(w), ctypes.c_int(int(bool(p.literal))),
                                 ctypes.c_int(FUSION_MODES.get(p.fusion, p.fusion)), _p(wf), _p(gS), _p(pts),
                                 _i64(pts.shape[0]), _p(gV), _nthreads(nthreads))
    _check(rc, "backward_at")
    return gV
