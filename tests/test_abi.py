"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/sal.h declares, and rejects bad arguments on the
host before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2201_06174_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(sal_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    declared = _declared()
    assert "sal_project" in declared and "sal_backward" in declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows each of them
    assert declared <= set(_lib.SIGNATURES), sorted(declared - set(_lib.SIGNATURES))


def test_version_and_grid_extent():
    lib = _lib.load()
    assert lib.sal_version().startswith(b"libsal")
    assert lib.sal_grid_extent(600, 2) == 300 and lib.sal_grid_extent(7, 3) == 3 and lib.sal_grid_extent(0, 2) == 0


def _err(rc):
    return _lib.STATUS_NAMES[rc]


@pytest.mark.parametrize("n,s,window,prec,shape,code", [
    (10, 1, 0, 0, (32, 32, 32), "SAL_ERR_UNSUPPORTED"),   # valid for the method, not built
    (7, 1, 0, 0, (32, 32, 32), "SAL_ERR_ARG"),            # odd side
    (8, 4, 0, 0, (32, 32, 32), "SAL_ERR_ARG"),            # overlap not above 50 %
    (8, 0, 0, 0, (32, 32, 32), "SAL_ERR_ARG"),
    (8, 1, 5, 0, (32, 32, 32), "SAL_ERR_ARG"),            # window
    (8, 1, 0, 9, (32, 32, 32), "SAL_ERR_ARG"),            # precision
    (16, 2, 0, 0, (7, 32, 32), "SAL_ERR_SHAPE"),          # axis shorter than n/2
    (8, 1, 0, 0, (32, 0, 32), "SAL_ERR_SHAPE"),           # empty volume
])
def test_project_rejects_bad_spec(n, s, window, prec, shape, code):
    lib = _lib.load()
    sp = _lib.SalSpec(n, s, window, prec)
    rc = lib.sal_project(ctypes.c_void_p(16), shape[0], shape[1], shape[2], sp, ctypes.c_void_p(16), None)
    assert _err(rc) == code
    assert lib.sal_last_error()


def test_null_buffers_rejected():
    lib = _lib.load()
    sp = _lib.SalSpec(8, 1, 0, 0)
    assert _err(lib.sal_project(None, 32, 32, 32, sp, ctypes.c_void_p(16), None)) == "SAL_ERR_ARG"
    assert _err(lib.sal_project(ctypes.c_void_p(16), 32, 32, 32, None, ctypes.c_void_p(16), None)) == "SAL_ERR_ARG"


def test_stencil_validation():
    lib = _lib.load()
    E, S = ctypes.c_void_p(16), ctypes.c_void_p(32)
    st, keep = _lib.make_stencil([[1, 0, 0]])
    assert _err(lib.sal_center_surround(E, 4, 4, 4, 2, st, S, None)) == "SAL_ERR_ARG"  # off the stride-2 grid
    st, keep = _lib.make_stencil([[0, 0, 0]])
    assert _err(lib.sal_center_surround(E, 4, 4, 4, 1, st, S, None)) == "SAL_ERR_ARG"  # no direction
    st, keep = _lib.make_stencil(np.ones((65, 3)))
    assert _err(lib.sal_center_surround(E, 4, 4, 4, 1, st, S, None)) == "SAL_ERR_ARG"  # too many
    st, keep = _lib.make_stencil([[1, 0, 0]])
    assert _err(lib.sal_center_surround(E, 4, 4, 4, 1, st, E, None)) == "SAL_ERR_ARG"  # aliasing


def test_empty_work_is_a_no_op():
    """Zero centres and an empty grid are valid and launch nothing (no device needed)."""
    lib = _lib.load()
    sp = _lib.SalSpec(8, 1, 0, 0)
    assert _err(lib.sal_local_spectra(None, 32, 32, 32, sp, None, 0, None, None)) == "SAL_OK"
    assert _err(lib.sal_local_spectra(None, 32, 32, 32, sp, None, -1, None, None)) == "SAL_ERR_ARG"
    st, keep = _lib.make_stencil([[1, 0, 0], [-1, 0, 0]])
    E, S = ctypes.c_void_p(16), ctypes.c_void_p(32)
    assert _err(lib.sal_center_surround(E, 0, 4, 4, 1, st, S, None)) == "SAL_OK"
    assert _err(lib.sal_center_surround(E, -1, 4, 4, 1, st, S, None)) == "SAL_ERR_SHAPE"


def test_fuse_validation():
    lib = _lib.load()
    p = ctypes.c_void_p(64)
    f = _lib.make_fusion("adapt_ls")
    # ADAPT_LS without a desired map
    assert _err(lib.sal_fuse(p, 4, 4, 4, f, None, None, 8, 8, 8, 2, p, p, p, 1 << 20, None)) == "SAL_ERR_ARG"
    # grid extents inconsistent with the volume
    f = _lib.make_fusion("equal")
    assert _err(lib.sal_fuse(p, 4, 4, 5, f, None, None, 8, 8, 8, 2, p, p, None, 0, None)) == "SAL_ERR_SHAPE"
    # workspace too small
    f = _lib.make_fusion("adapt_ls")
    assert _err(lib.sal_fuse(p, 4, 4, 4, f, p, None, 8, 8, 8, 2, p, p, p, 8, None)) == "SAL_ERR_NOMEM"
    f = _lib.make_fusion("adapt_ls", delta=-1.0)
    assert _err(lib.sal_fuse(p, 4, 4, 4, f, p, None, 8, 8, 8, 2, p, p, p, 1 << 20, None)) == "SAL_ERR_ARG"
    f = _lib.make_fusion(7)
    assert _err(lib.sal_fuse(p, 4, 4, 4, f, p, None, 8, 8, 8, 2, p, p, p, 1 << 20, None)) == "SAL_ERR_ARG"


def test_python_binding_refuses_cpu_tensors():
    import torch
    import paper_2201_06174_amd as sal
    with pytest.raises(TypeError):
        sal.project(torch.zeros(8, 8, 8), 8, 1)


def test_peak_microbenchmark_arguments():
    lib = _lib.load()
    # flops of one launch: waves x iters x chains x flops per instruction
    assert lib.sal_peak_compute_flops(0, 100, 10) == 10 * 4 * 100 * 4 * 2048
    assert lib.sal_peak_compute_flops(1, 100, 10) == 10 * 4 * 100 * 4 * 32768
    assert lib.sal_peak_compute_flops(2, 100, 10) == 10 * 4 * 100 * 4 * 32768
    assert lib.sal_peak_compute_flops(3, 100, 10) == 10 * 256 * 100 * 8 * 2
    assert lib.sal_peak_compute_flops(4, 100, 10) == 0 and lib.sal_peak_compute_flops(0, 16385, 10) == 0
    fake = ctypes.c_void_p(256)
    for kind, iters, blocks in [(4, 10, 10), (-1, 10, 10), (0, 0, 10), (0, 16385, 10), (0, 10, 0), (0, 10, 1 << 21)]:
        assert _err(lib.sal_peak_compute(kind, iters, blocks, fake, None)) == "SAL_ERR_ARG"
    assert _err(lib.sal_peak_compute(0, 10, 10, None, None)) == "SAL_ERR_ARG"
    big = ctypes.c_void_p(1 << 20)
    for kind, src, dst, nbytes in [(2, fake, big, 1024), (0, fake, None, 1000), (0, fake, None, 0),
                                   (0, ctypes.c_void_p(264), None, 1024), (1, fake, None, 1024),
                                   (1, fake, ctypes.c_void_p(256 + 512), 1024)]:
        assert _err(lib.sal_peak_stream(kind, src, dst, nbytes, fake, 16, None)) == "SAL_ERR_ARG"


def test_per_plane_stencil_validation():
    lib = _lib.load()
    E, S = ctypes.c_void_p(16), ctypes.c_void_p(32)
    ok = ([[1, 0, 0], [-1, 0, 0]], None)
    # an empty grid launches nothing, so a valid per-plane stencil returns OK without a device
    st, keep = _lib.make_stencil(None, planes=[ok, ([[0, 0, 2]], [0.5]), ([[2, 2, 0]], None)])
    assert _err(lib.sal_center_surround(E, 0, 4, 4, 1, st, S, None)) == "SAL_OK"
    # one plane off the stride-2 grid
    st, keep = _lib.make_stencil(None, planes=[ok, ([[0, 0, 2]], None), ([[2, 2, 0]], None)])
    assert _err(lib.sal_center_surround(E, 0, 4, 4, 2, st, S, None)) == "SAL_ERR_ARG"
    # the union of the three planes holds more than SAL_MAX_STENCIL distinct offsets
    many = [np.array([[a + 1, b, c] for a in range(4) for b in range(4) for c in range(2)]) + 10 * m
            for m in range(3)]
    st, keep = _lib.make_stencil(None, planes=[(o, None) for o in many])
    assert _err(lib.sal_center_surround(E, 0, 4, 4, 1, st, S, None)) == "SAL_ERR_ARG"
    # a per-plane stencil may not nest further stencils
    st, keep = _lib.make_stencil(None, planes=[ok, ok, ok])
    inner = ctypes.cast(st.per_plane, ctypes.POINTER(_lib.SalStencil))
    inner[1].per_plane = st.per_plane
    assert _err(lib.sal_center_surround(E, 0, 4, 4, 1, st, S, None)) == "SAL_ERR_ARG"


def test_sections_and_groups():
    lib = _lib.load()
    f = _lib.make_fusion("adapt_ls", sections=3)
    assert lib.sal_fuse_groups(f, 7) == 3 and lib.sal_fuse_groups(f, 6) == 2 and lib.sal_fuse_groups(f, 0) == 0
    assert lib.sal_fuse_groups(_lib.make_fusion("equal"), 200) == 1 and lib.sal_fuse_groups(None, 5) == 0
    # the workspace grows with the number of groups
    one = lib.sal_fuse_workspace_size(4, 9, 4, _lib.make_fusion("adapt_ls"))
    assert lib.sal_fuse_workspace_size(4, 9, 4, f) == 3 * one
    sp = _lib.SalSpec(8, 1, 0, 0)
    assert lib.sal_backward_workspace_size(16, 18, 16, sp, f) > lib.sal_backward_workspace_size(16, 18, 16, sp, None)
    p = ctypes.c_void_p(64)
    bad = _lib.make_fusion("equal", sections=-1)
    assert _err(lib.sal_fuse(p, 4, 4, 4, bad, None, None, 8, 8, 8, 2, p, p, None, 0, None)) == "SAL_ERR_ARG"
    # workspace sized for one group is too small for three
    assert _err(lib.sal_fuse(p, 4, 9, 4, f, p, None, 8, 18, 8, 2, p, p, p, one, None)) == "SAL_ERR_NOMEM"


def test_line_template_matches_the_oracle():
    """sal_line_template (host code of the library) and the oracle's own template give the
    same offsets and weights (the two are written independently)."""
    from oracle import oracle as orc
    for d, L, sig in (([2, 0, 0], 3, 1.5), ([0, 0, 1], 1, 0.5), ([1, 0, 1], 4, 2.0), ([0, -3, 3], 2, 1.0)):
        off, w = _lib.line_template(d, L, sig)
        ro, rw = orc.line_template(d, L, sig)
        assert np.array_equal(off, ro)
        assert np.allclose(w, rw, rtol=1e-7, atol=0)
    for d, L, sig in (([0, 0, 0], 2, 1.0), ([1, 0, 0], 0, 1.0), ([1, 0, 0], 33, 1.0), ([1, 0, 0], 2, 0.0)):
        with pytest.raises(_lib.SalError):
            _lib.line_template(d, L, sig)


def test_plan_status_arguments():
    lib = _lib.load()
    c, f = ctypes.c_int64(), ctypes.c_int64()
    assert _err(lib.sal_plan_status(None, None, ctypes.byref(c), ctypes.byref(f))) == "SAL_ERR_ARG"


def test_sequential_fusion_validation():
    lib = _lib.load()
    p = ctypes.c_void_p(64)
    ws = 1 << 24

    def fuse(f, D=p):
        return _err(lib.sal_fuse(p, 4, 4, 4, f, D, None, 8, 8, 8, 2, p, p, p, ws, None))
    assert fuse(_lib.make_fusion("nlms", mu=0.5), None) == "SAL_ERR_ARG"     # no desired map
    assert fuse(_lib.make_fusion("lms", mu=0.0)) == "SAL_ERR_ARG"            # no step
    assert fuse(_lib.make_fusion("nlms", mu=0.5, eps=-1.0)) == "SAL_ERR_ARG"
    assert fuse(_lib.make_fusion("rls", delta=1.0, lam=1.5)) == "SAL_ERR_ARG"  # forgetting factor above 1
    assert fuse(_lib.make_fusion("rls", delta=0.0)) == "SAL_ERR_ARG"          # P0 undefined
    assert fuse(_lib.make_fusion("nlms", mu=0.5, passes=0)) == "SAL_ERR_ARG"
    f = _lib.make_fusion("nlms", mu=0.5)
    # the workspace holds the index list of the grid's points
    assert lib.sal_fuse_workspace_size(4, 4, 4, f) >= 4 * 64
    assert _err(lib.sal_fuse(p, 4, 4, 4, f, p, None, 8, 8, 8, 2, p, p, p, 16, None)) == "SAL_ERR_NOMEM"
    assert _err(lib.sal_adapt_weights(p, 4, 4, 4, _lib.make_fusion("adapt_ls"), p, None, p, None, 0, None, p, ws,
                                      None)) == "SAL_ERR_ARG"
    assert _err(lib.sal_adapt_weights(p, 4, 4, 4, f, p, None, p, None, 5, None, p, ws, None)) == "SAL_ERR_ARG"
    # not taken by the adjoint, the no-allocation fusion and the plans
    sp = _lib.SalSpec(8, 1, 0, 0)
    st, keep = _lib.make_stencil([[1, 0, 0], [-1, 0, 0]])
    assert _err(lib.sal_backward(p, 8, 8, 8, sp, st, f, p, p, p, p, None, p, p, p, ws, None)) == "SAL_ERR_UNSUPPORTED"
    assert _err(lib.sal_fuse_noalloc(p, 4, 4, 4, f, p, None, 8, 8, 8, 2, p, p, None)) == "SAL_ERR_UNSUPPORTED"


def test_energy_feature_validation():
    lib = _lib.load()
    for prec, code in ((1, "SAL_ERR_UNSUPPORTED"), (2, "SAL_ERR_UNSUPPORTED")):
        sp = _lib.SalSpec(8, 1, 0, prec, 1)
        rc = lib.sal_project(ctypes.c_void_p(16), 32, 32, 32, sp, ctypes.c_void_p(16), None)
        assert _err(rc) == code
    sp = _lib.SalSpec(8, 1, 0, 0, 7)
    assert _err(lib.sal_project(ctypes.c_void_p(16), 32, 32, 32, sp, ctypes.c_void_p(16), None)) == "SAL_ERR_ARG"
