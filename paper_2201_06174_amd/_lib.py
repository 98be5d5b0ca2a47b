"""ctypes binding of libsal.so (the C ABI declared in include/sal.h).

Argument marshalling only.  The library must have been built
(``python -m paper_2201_06174_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsal.so")

SAL_OK = 0
STATUS_NAMES = {0: "SAL_OK", 1: "SAL_ERR_ARG", 2: "SAL_ERR_SHAPE", 3: "SAL_ERR_UNSUPPORTED", 4: "SAL_ERR_NOMEM",
                5: "SAL_ERR_DEVICE", 6: "SAL_ERR_STATE"}
WINDOW = {"hann": 0, "rect": 1}
PRECISION = {"fp32": 0, "split_bf16": 1, "fp16": 2}
FEATURE = {"magnitude": 0, "energy": 1}
FUSION = {"equal": 0, "fixed": 1, "adapt_ls": 2, "lms": 3, "nlms": 4, "rls": 5}
MAX_STENCIL = 64


class SalSpec(ctypes.Structure):
    _fields_ = [("n", c_int32), ("s", c_int32), ("window", c_int32), ("precision", c_int32), ("feature", c_int32)]


class SalStencil(ctypes.Structure):
    pass


SalStencil._fields_ = [("q", c_int32), ("offsets", POINTER(c_int32)), ("weights", POINTER(c_float)),
                       ("literal", c_int32), ("per_plane", POINTER(SalStencil))]


class SalFusion(ctypes.Structure):
    _fields_ = [("mode", c_int32), ("w_fixed", c_double * 3), ("delta", c_double), ("sections", c_int64),
                ("mu", c_double), ("eps", c_double), ("lambda_", c_double), ("passes", c_int32)]


class SalBatchItem(ctypes.Structure):
    _fields_ = [("V", c_void_p), ("T", c_int64), ("IL", c_int64), ("XL", c_int64), ("spec", SalSpec),
                ("stencil", SalStencil), ("fusion", SalFusion), ("D", c_void_p), ("mask", c_void_p),
                ("E_out", c_void_p), ("Sm_out", c_void_p), ("W_out", c_void_p), ("S_out", c_void_p)]


PLAN_AUTOTUNE = 1
PLAN_NO_GRAPH = 2


class SalError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


# name -> (restype, argtypes); every entry point of include/sal.h
SIGNATURES = {
    "sal_init": (c_int32, []),
    "sal_fuse_groups": (c_int64, [POINTER(SalFusion), c_int64]),
    "sal_line_template": (c_int32, [POINTER(c_int32), c_int32, c_double, POINTER(c_int32), POINTER(c_float)]),
    "sal_plan_status": (c_int32, [c_void_p, c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    "sal_last_error": (c_char_p, []),
    "sal_version": (c_char_p, []),
    "sal_grid_extent": (c_int64, [c_int64, c_int32]),
    "sal_local_spectra": (c_int32, [c_void_p, c_int64, c_int64, c_int64, POINTER(SalSpec), c_void_p, c_int64, c_void_p,
                                    c_void_p]),
    "sal_project": (c_int32, [c_void_p, c_int64, c_int64, c_int64, POINTER(SalSpec), c_void_p, c_void_p]),
    "sal_center_surround": (c_int32, [c_void_p, c_int64, c_int64, c_int64, c_int32, POINTER(SalStencil), c_void_p,
                                      c_void_p]),
    "sal_fuse_workspace_size": (c_size_t, [c_int64, c_int64, c_int64, POINTER(SalFusion)]),
    "sal_fuse": (c_int32, [c_void_p, c_int64, c_int64, c_int64, POINTER(SalFusion), c_void_p, c_void_p, c_int64,
                           c_int64, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "sal_adapt_weights": (c_int32, [c_void_p, c_int64, c_int64, c_int64, POINTER(SalFusion), c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]),
    "sal_fuse_noalloc_max_bytes": (c_size_t, []),
    "sal_fuse_noalloc": (c_int32, [c_void_p, c_int64, c_int64, c_int64, POINTER(SalFusion), c_void_p, c_void_p,
                                   c_int64, c_int64, c_int64, c_int32, c_void_p, c_void_p, c_void_p]),
    "sal_backward_workspace_size": (c_size_t, [c_int64, c_int64, c_int64, POINTER(SalSpec), POINTER(SalFusion)]),
    "sal_backward": (c_int32, [c_void_p, c_int64, c_int64, c_int64, POINTER(SalSpec), POINTER(SalStencil),
                               POINTER(SalFusion), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_size_t, c_void_p]),
    "sal_plan_create": (c_int32, [POINTER(SalBatchItem), c_int64, ctypes.c_uint32, POINTER(c_void_p)]),
    "sal_plan_launch": (c_int32, [c_void_p, c_void_p]),
    "sal_plan_describe": (c_char_p, [c_void_p]),
    "sal_plan_destroy": (c_int32, [c_void_p]),
    # device throughput microbenchmarks (include/sal_peak.h)
    "sal_peak_compute_flops": (c_int64, [c_int32, c_int64, c_int64]),
    "sal_peak_compute": (c_int32, [c_int32, c_int64, c_int64, c_void_p, c_void_p]),
    "sal_peak_stream": (c_int32, [c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p]),
}

_lib = None


def load():
    """Load libsal.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsal.so is not built (run `python -m paper_2201_06174_amd.build`)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if not hasattr(lib, name):
                continue
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    lib = load()
    return [name for name in SIGNATURES if hasattr(lib, name)]


def check(rc):
    if rc != SAL_OK:
        msg = load().sal_last_error()
        raise SalError(rc, msg.decode() if msg else "")


def _fill_stencil(st, offsets, weights, literal):
    import numpy as np
    off = np.ascontiguousarray(offsets, dtype=np.int32).reshape(-1, 3)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32).reshape(-1)
    if w is not None and w.shape[0] != off.shape[0]:
        raise ValueError("one weight per offset: %d offsets, %d weights" % (off.shape[0], w.shape[0]))
    st.q = off.shape[0]
    st.offsets = off.ctypes.data_as(POINTER(c_int32))
    st.weights = w.ctypes.data_as(POINTER(c_float)) if w is not None else POINTER(c_float)()
    st.literal = 1 if literal else 0
    st.per_plane = POINTER(SalStencil)()
    return (off, w)


def make_stencil(offsets, weights=None, literal=False, planes=None):
    """SalStencil plus the host arrays it points to (keep both alive).  planes: None, or
    [(offsets, weights or None)] for the planes t, x, y (per-plane stencils)."""
    st = SalStencil()
    if planes is None:
        return st, _fill_stencil(st, offsets, weights, literal)
    if len(planes) != 3:
        raise ValueError("one stencil per plane (t, x, y)")
    arr = (SalStencil * 3)()
    keep = [arr]
    for m, (off, w) in enumerate(planes):
        keep.append(_fill_stencil(arr[m], off, w, literal))
    st.q = 0
    st.offsets = POINTER(c_int32)()
    st.weights = POINTER(c_float)()
    st.literal = 1 if literal else 0
    st.per_plane = ctypes.cast(arr, POINTER(SalStencil))
    return st, keep


def make_fusion(mode="equal", wfix=None, delta=0.0, sections=0, mu=0.0, eps=0.0, lam=1.0, passes=1):
    """SalFusion; wfix: FIXED weights, or the starting weights of LMS / NLMS / RLS."""
    f = SalFusion()
    f.mode = FUSION[mode] if isinstance(mode, str) else int(mode)
    w = [0.0, 0.0, 0.0] if wfix is None else [float(v) for v in wfix]
    f.w_fixed = (c_double * 3)(*w)
    f.delta = float(delta)
    f.sections = int(sections)
    f.mu = float(mu)
    f.eps = float(eps)
    f.lambda_ = float(lam)
    f.passes = int(passes)
    return f


def line_template(direction, length, sigma):
    """(offsets [2L][3] int32, weights [2L] float32) of sal_line_template (host only)."""
    import numpy as np
    d = np.ascontiguousarray(direction, dtype=np.int32).reshape(3)
    off = np.zeros((2 * int(length), 3), np.int32)
    w = np.zeros(2 * int(length), np.float32)
    check(load().sal_line_template(d.ctypes.data_as(POINTER(c_int32)), int(length), float(sigma),
                                   off.ctypes.data_as(POINTER(c_int32)), w.ctypes.data_as(POINTER(c_float))))
    return off, w


def make_spec(n, s, window="hann", precision="fp32", feature="magnitude"):
    sp = SalSpec()
    sp.n, sp.s = int(n), int(s)
    sp.window = WINDOW[window] if isinstance(window, str) else int(window)
    sp.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    sp.feature = FEATURE[feature] if isinstance(feature, str) else int(feature)
    return sp
