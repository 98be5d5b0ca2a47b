"""sal_fuse_noalloc (the fusion with its workspace in the library's static device array)
against sal_fuse with a caller-allocated workspace, through the C ABI: two calls in a
row, the second on a smaller grid, every output bit for bit; sizes beyond the static
array are refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_06174_amd as sal
    from paper_2201_06174_amd import _lib
    sal.init()
    return torch, sal, _lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _both(torch, sal, _lib, shape, s, mode, sections, seed, masked):
    lib = _lib.load()
    rng = np.random.default_rng(seed)
    gs = sal.grid_shape(shape, s)
    Sm = torch.from_numpy(rng.uniform(0.1, 2.0, size=(3,) + gs).astype(np.float32)).cuda()
    D = torch.from_numpy(rng.uniform(size=gs).astype(np.float32)).cuda()
    mask = torch.from_numpy((rng.uniform(size=gs) < 0.6).astype(np.uint8)).cuda() if masked else None
    f = _lib.make_fusion(mode, (0.2, 0.5, 0.3), 1e-6, sections)
    K = int(lib.sal_fuse_groups(f, gs[1]))
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = []
    for noalloc in (False, True):
        W = torch.full((K, 4), float("nan"), dtype=torch.float64, device="cuda")
        S = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
        if noalloc:
            rc = lib.sal_fuse_noalloc(_p(Sm), gs[0], gs[1], gs[2], f, _p(D), _p(mask), shape[0], shape[1], shape[2],
                                      s, _p(W), _p(S), st)
        else:
            nb = int(lib.sal_fuse_workspace_size(gs[0], gs[1], gs[2], f))
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            rc = lib.sal_fuse(_p(Sm), gs[0], gs[1], gs[2], f, _p(D), _p(mask), shape[0], shape[1], shape[2], s,
                              _p(W), _p(S), _p(ws), nb, st)
        _lib.check(rc)
        torch.cuda.synchronize()
        out.append((W, S))
    return out, K


def test_fuse_noalloc_matches_fuse(torch_lib):
    torch, sal, _lib = torch_lib
    print("sal_fuse_noalloc: two calls in a row, the second smaller", flush=True)
    # the first call fills 33 weight groups of the scratch, the second (smaller, one group)
    # must not see anything of it
    for shape, s, mode, sections, seed, masked in (((40, 66, 36), 2, "adapt_ls", 1, 1, True),
                                                   ((12, 9, 10), 1, "adapt_ls", 0, 2, False)):
        (ref, got), K = _both(torch, sal, _lib, shape, s, mode, sections, seed, masked)
        print("  grid of %s, stride %d, %d weight groups" % (shape, s, K), flush=True)
        assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
        assert not torch.isnan(got[1]).any()
    # the other fusion modes need no scratch
    for mode in ("equal", "fixed"):
        (ref, got), _ = _both(torch, sal, _lib, (9, 20, 7), 1, mode, 3, 3, False)
        assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])


def test_fuse_noalloc_refuses_more_groups_than_its_scratch(torch_lib):
    torch, sal, _lib = torch_lib
    lib = _lib.load()
    gs, shape = (4, 65, 4), (4, 65, 4)
    f = _lib.make_fusion("adapt_ls", None, 0.0, 1)  # 65 groups of one inline section
    Sm = torch.zeros((3,) + gs, dtype=torch.float32, device="cuda")
    D = torch.zeros(gs, dtype=torch.float32, device="cuda")
    W = torch.empty((65, 4), dtype=torch.float64, device="cuda")
    S = torch.empty(shape, dtype=torch.float32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.sal_fuse_noalloc(_p(Sm), 4, 65, 4, f, _p(D), None, 4, 65, 4, 1, _p(W), _p(S), st)
    assert _lib.STATUS_NAMES[rc] == "SAL_ERR_NOMEM" and b"64 groups" in lib.sal_last_error()
    assert lib.sal_fuse_noalloc_max_bytes() == 64 * (256 * 11 + 16) * 8
